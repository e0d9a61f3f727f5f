// mer_raster.hip -- triangle set-up, tile binning and the tiled z-buffer
// rasterizer with barycentric/depth resolve (supplement, "Rasterization
// module" and "Barycentrics module").
//
// Pipeline for one mer_rasterize call over all views:
//   k_prep      per-view prefix tables (triangles, tiles), clear tile counters
//   k_setup     one thread per (view, triangle): snap, cull; a triangle whose
//               box of pixel centres is small is rasterized right there
//               (coverage + depth key + 64-bit atomic max into the per-pixel
//               key); a larger one gets a 64-byte coverage record, its box,
//               and counts the tiles it overlaps
//   k_scan_*    exclusive scan of tile counts -> bin offsets
//   k_fill      one thread per (view, triangle): write its record index into
//               every overlapped tile's list
//   k_raster    one workgroup per tile, one lane per pixel: start from the
//               pixel's key, stage the tile's records in LDS, exact coverage,
//               binary32 depth key, 64-bit (1/z, ~id) max; then resolve the
//               winner's depth and barycentrics from its vertices
// The (1/z, ~id) maximum does not depend on the order in which candidates
// arrive, so both paths and any tile shape give the same index image.
#include "mer_internal.h"

namespace mer {

// ----------------------------------------------------------------- prep
// Block-wide exclusive scan over n values (any n); one block of 1024 threads.
__global__ void __launch_bounds__(1024) k_prep(const mer_view* __restrict__ views, int n_views, int tw_log2,
                                               int th_log2, long long* __restrict__ tri_base,
                                               long long* __restrict__ tile_base, long long* __restrict__ status) {
  __shared__ long long s_tri[1024], s_tile[1024];
  const int tid = threadIdx.x;
  const int per = (n_views + 1023) / 1024;
  const int lo = tid * per, hi = min(n_views, lo + per);
  long long a = 0, b = 0;
  for (int i = lo; i < hi; ++i) {
    const mer_view vw = views[i];
    a += vw.n_t;
    b += (long long)((vw.W + (1 << tw_log2) - 1) >> tw_log2) * ((vw.H + (1 << th_log2) - 1) >> th_log2);
  }
  s_tri[tid] = a;
  s_tile[tid] = b;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    long long x = tid >= off ? s_tri[tid - off] : 0, y = tid >= off ? s_tile[tid - off] : 0;
    __syncthreads();
    s_tri[tid] += x;
    s_tile[tid] += y;
    __syncthreads();
  }
  long long ea = s_tri[tid] - a, eb = s_tile[tid] - b;  // exclusive prefix of this thread's chunk
  for (int i = lo; i < hi; ++i) {
    const mer_view vw = views[i];
    tri_base[i] = ea;
    tile_base[i] = eb;
    ea += vw.n_t;
    eb += (long long)((vw.W + (1 << tw_log2) - 1) >> tw_log2) * ((vw.H + (1 << th_log2) - 1) >> th_log2);
  }
  if (tid == 1023) {
    tri_base[n_views] = s_tri[1023];
    tile_base[n_views] = s_tile[1023];
  }
  if (status && tid < 8) status[tid] = 0;
}

__global__ void k_zero_i32(int* __restrict__ p, long long n) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    p[i] = 0;
}

__global__ void k_zero_u64(unsigned long long* __restrict__ p, long long n) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    p[i] = 0ull;
}

// ---------------------------------------------------------------- setup
struct BBox {
  short x0, y0, x1, y1;  // inclusive pixel range; x0 > x1 when empty/culled
};

// Triangles whose box spans more than big_tiles tiles (a plan setting) are
// listed by the count pass and binned by k_bin_big, where a whole wave walks
// one triangle's tiles 64 at a time: a few large triangles then do not hold
// every lane of their wave in a long loop.

__device__ __forceinline__ int box_tiles(const BBox& bb, int tw_log2, int th_log2) {
  return ((bb.x1 >> tw_log2) - (bb.x0 >> tw_log2) + 1) * ((bb.y1 >> th_log2) - (bb.y0 >> th_log2) + 1);
}

// The box's tile k (row-major) and the part of the box inside it; f(global
// tile) when box_may_cover accepts it -- the one test of every binning pass.
template <typename F>
__device__ __forceinline__ void box_tile_test(const Rec& R, const BBox& bb, int tiles_x, long long base, int tw_log2,
                                              int th_log2, int tx, int ty, F f) {
  const int bx0 = max(tx << tw_log2, (int)bb.x0), bx1 = min(((tx + 1) << tw_log2) - 1, (int)bb.x1);
  const int by0 = max(ty << th_log2, (int)bb.y0), by1 = min(((ty + 1) << th_log2) - 1, (int)bb.y1);
  if (box_may_cover(R, bx0, by0, bx1, by1)) f((int)(base + (long long)ty * tiles_x + tx));
}

template <typename F>
__device__ __forceinline__ void for_each_tile(const Rec& R, const BBox& bb, int W, long long base, int tw_log2,
                                              int th_log2, F f) {
  const int tiles_x = (W + (1 << tw_log2) - 1) >> tw_log2;
  for (int ty = bb.y0 >> th_log2; ty <= (bb.y1 >> th_log2); ++ty)
    for (int tx = bb.x0 >> tw_log2; tx <= (bb.x1 >> tw_log2); ++tx)
      box_tile_test(R, bb, tiles_x, base, tw_log2, th_log2, tx, ty, f);
}

// A whole wave over one (wave-uniform) triangle's tiles, lane k taking tiles
// k, k + 64, ...
template <typename F>
__device__ __forceinline__ void wave_each_tile(const Rec& R, const BBox& bb, int W, long long base, int tw_log2,
                                               int th_log2, F f) {
  const int tiles_x = (W + (1 << tw_log2) - 1) >> tw_log2;
  const int tx0 = bb.x0 >> tw_log2, ty0 = bb.y0 >> th_log2, ntx = (bb.x1 >> tw_log2) - tx0 + 1;
  const int nt = box_tiles(bb, tw_log2, th_log2);
  for (int k = threadIdx.x & 63; k < nt; k += 64)
    box_tile_test(R, bb, tiles_x, base, tw_log2, th_log2, tx0 + k % ntx, ty0 + k / ntx, f);
}

// Tiles of a box of at most 16 tiles whose test passed, as a 16-bit mask
// over the box's tiles in row-major order (the count pass stores it in bits
// 16-31 of the record's tl word, with bit 4 set): the fill pass walks the
// set bits instead of testing every tile again.
constexpr int kMaskValid = 16;
template <typename F>
__device__ __forceinline__ void for_each_masked_tile(unsigned m, const BBox& bb, int W, long long base, int tw_log2,
                                                     int th_log2, F f) {
  const int tiles_x = (W + (1 << tw_log2) - 1) >> tw_log2;
  const int tx0 = bb.x0 >> tw_log2, ty0 = bb.y0 >> th_log2, ntx = (bb.x1 >> tw_log2) - tx0 + 1;
  const unsigned inv = (256u + (unsigned)ntx - 1u) / (unsigned)ntx;  // k / ntx = (k inv) >> 8 for k < 16, ntx <= 16
  while (m) {
    const int k = __builtin_ctz(m);
    m &= m - 1u;
    const int dy = (int)(((unsigned)k * inv) >> 8), dx = k - dy * ntx;
    f((int)(base + (long long)(ty0 + dy) * tiles_x + tx0 + dx));
  }
}

// Workgroup table of tile counters: the count and fill passes add into LDS
// and touch each tile's global counter once per workgroup (a workgroup of
// large triangles can meet thousands of tiles; tiles the table does not take
// use their global counter directly).  A key lives in a window of kBinProbe
// slots from its hash; slots go from empty to a key once and never change
// again.
constexpr int kBinLog2 = 10;    // table of 2^kBinLog2 tile slots
constexpr int kBinSlots = 1 << kBinLog2;
constexpr int kBinFull = kBinSlots * 3 / 4;
constexpr int kBinProbe = 16;

__device__ __forceinline__ void clear_tile_table(int* s_tkey, int* s_tcnt, int* s_nocc) {
  for (int i = threadIdx.x; i < kBinSlots; i += blockDim.x) {
    s_tkey[i] = -1;
    s_tcnt[i] = 0;
  }
  if (threadIdx.x == 0) *s_nocc = 0;
}

// Slot of tile `key`, inserting it if INSERT; -1 if absent.
//
// Without CUTOFF a key is refused only when every slot of its window holds
// another key.  That cannot change later, and a key once in the table stays
// there, so an inserting lookup and a later frozen lookup (INSERT = false,
// after a barrier) of the same key always agree.  The fill pass depends on
// this: its two passes must make the same decision for every entry, or an
// entry counted outside the workgroup's range would be written inside it.
//
// CUTOFF also refuses a new key once 3/4 of the slots are taken, which keeps
// probe windows short; the decision then depends on timing (a lane can be
// refused at an empty slot that another lane fills with the same key a
// moment later), so it is only for the count pass, where a refused entry is
// simply counted in global memory instead.
template <bool INSERT, bool CUTOFF>
__device__ __forceinline__ int tile_slot(int* s_tkey, int* s_nocc, int key) {
  const unsigned h = ((unsigned)key * 2654435761u) >> (32 - kBinLog2);
#pragma unroll 1
  for (int probe = 0; probe < kBinProbe; ++probe) {
    const int sl = (int)((h + probe) & (kBinSlots - 1));
    const int cur = s_tkey[sl];
    if (cur == key) return sl;
    if (cur == -1) {
      if (!INSERT || (CUTOFF && *s_nocc >= kBinFull)) return -1;
      const int old = atomicCAS(&s_tkey[sl], -1, key);
      if (old == -1) {
        if (CUTOFF) atomicAdd(s_nocc, 1);
        return sl;
      }
      if (old == key) return sl;
    }
  }
  return -1;
}

__global__ void __launch_bounds__(kBinBlock) k_setup(const mer_view* __restrict__ views, int n_views,
                                               const float* __restrict__ v, const int32_t* __restrict__ tri,
                                               const long long* __restrict__ tri_base,
                                               const long long* __restrict__ tile_base, long long total_tris,
                                               int tw_log2, int th_log2, int small_px, int big_tiles,
                                               long long px_begin,
                                               Rec* __restrict__ rec, BBox* __restrict__ bbox,
                                               int* __restrict__ count, unsigned long long* __restrict__ key,
                                               long long* __restrict__ status, int* __restrict__ big,
                                               int* __restrict__ big_n) {
  __shared__ int s_tkey[kBinSlots], s_tcnt[kBinSlots], s_nocc;
  __shared__ int s_big[kBinBlock], s_nbig;
  clear_tile_table(s_tkey, s_tcnt, &s_nocc);
  if (threadIdx.x == 0) s_nbig = 0;
  __syncthreads();
  const long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  bool culled = false;
  if (g < total_tris) {
    const int vi = wave_bucket(tri_base, n_views, g);
    const mer_view vw = views[vi];
    const long long t = g - tri_base[vi];
    const Snap s = snap_triangle(v, vw, tri_row(tri, vw, (int)t));
    BBox bb = {1, 1, 0, 0};
    if (!s.ok) {
      culled = true;
    } else {
      const Rec R = make_rec(s);
      int xmin = min(s.X[0], min(s.X[1], s.X[2])), xmax = max(s.X[0], max(s.X[1], s.X[2]));
      int ymin = min(s.Y[0], min(s.Y[1], s.Y[2])), ymax = max(s.Y[0], max(s.Y[1], s.Y[2]));
      // pixel centres 256 p + 128 within [min, max]: p in [ceil((min-128)/256), floor((max-128)/256)]
      int pxa = -((-(xmin - 128)) >> 8), pxb = (xmax - 128) >> 8;
      int pya = -((-(ymin - 128)) >> 8), pyb = (ymax - 128) >> 8;
      pxa = max(pxa, 0);
      pya = max(pya, 0);
      pxb = min(pxb, vw.W - 1);
      pyb = min(pyb, vw.H - 1);
      if (pxa <= pxb && pya <= pyb && (pxb - pxa + 1) * (pyb - pya + 1) <= small_px) {
        // small triangle: rasterize its few pixel centres here
        unsigned long long* kv = key + (vw.px_off - px_begin);
        const long long dx0 = (long long)R.A[0] * 256, dx1 = (long long)R.A[1] * 256, dx2 = (long long)R.A[2] * 256;
        for (int y = pya; y <= pyb; ++y) {
          long long E[3];
          edge_eval(R, pxa, y, E);  // then step along the row: E += 256 A
          for (int x = pxa; x <= pxb; ++x) {
            if (covered(E)) {
              float e[3], d;
              edge_values(R, E, e, d);
              atomicMax(kv + (long long)y * vw.W + x, vis_key(depth_key(R, e, d), (int)t));
            }
            E[0] += dx0;
            E[1] += dx1;
            E[2] += dx2;
          }
        }
      } else if (pxa <= pxb && pya <= pyb) {
        Rec Rm = R;
        bb.x0 = (short)pxa;
        bb.x1 = (short)pxb;
        bb.y0 = (short)pya;
        bb.y1 = (short)pyb;
        const int nb = box_tiles(bb, tw_log2, th_log2);
        if (nb > big_tiles) {
          s_big[atomicAdd(&s_nbig, 1)] = (int)g;  // counted by k_bin_big
        } else {
          const int tiles_x = (vw.W + (1 << tw_log2) - 1) >> tw_log2;
          const long long base = tile_base[vi];
          unsigned mask = 0u;
          int k = 0;
          for (int ty = bb.y0 >> th_log2; ty <= (bb.y1 >> th_log2); ++ty)
            for (int tx = bb.x0 >> tw_log2; tx <= (bb.x1 >> tw_log2); ++tx, ++k)
              box_tile_test(R, bb, tiles_x, base, tw_log2, th_log2, tx, ty, [&](int gt) {
                mask |= k < 16 ? 1u << k : 0u;
                const int sl = tile_slot<true, true>(s_tkey, &s_nocc, gt);
                if (sl >= 0) atomicAdd(&s_tcnt[sl], 1);
                else atomicAdd(count + gt, 1);
              });
          if (nb <= 16) Rm.tl |= kMaskValid | (int)(mask << 16);
        }
        rec[g] = Rm;
      }
    }
    bbox[g] = bb;
  }
  __syncthreads();
  // one global atomic per (workgroup, tile); this workgroup's list of large
  // triangles goes to its own slot of the list
  for (int i = threadIdx.x; i < kBinSlots; i += blockDim.x)
    if (s_tkey[i] >= 0) atomicAdd(count + s_tkey[i], s_tcnt[i]);
  const int nbig = s_nbig;
  for (int i = threadIdx.x; i < nbig; i += blockDim.x) big[(long long)blockIdx.x * kBinBlock + i] = s_big[i];
  if (threadIdx.x == 0) big_n[blockIdx.x] = nbig;
  // one atomic per wave for the culled count
  unsigned long long m = __ballot(culled);
  if (m && (threadIdx.x & 63) == __ffsll((long long)m) - 1) atomicAdd((unsigned long long*)status + 1, (unsigned long long)__popcll(m));
}

// ----------------------------------------------------------------- scan
// Exclusive scan of count[0..n) into offs[0..n], offs[n] = total, in 64-bit
// with offsets saturated at INT_MAX: the bin pool is smaller than that, so a
// tile whose range does not fit takes the raster's overflow path.  Blocks of
// 256 threads x 4 items.
__device__ __forceinline__ long long wave_incl_scan(long long x) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const long long y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  return x;
}

__device__ __forceinline__ long long block_excl_scan_256(long long x, long long* s_wave, long long& total) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const long long inc = wave_incl_scan(x);
  if (lane == 63) s_wave[w] = inc;
  __syncthreads();
  long long pre = 0;
  for (int i = 0; i < w; ++i) pre += s_wave[i];
  total = s_wave[0] + s_wave[1] + s_wave[2] + s_wave[3];
  __syncthreads();
  return pre + inc - x;
}

__device__ __forceinline__ int sat_int(long long x) { return x > 2147483647ll ? 2147483647 : (int)x; }

__global__ void __launch_bounds__(256) k_scan_partial(const int* __restrict__ count, long long n,
                                                      long long* __restrict__ part) {
  __shared__ long long s_wave[4];
  const long long base = (long long)blockIdx.x * 1024 + threadIdx.x * 4;
  long long s = 0;
#pragma unroll
  for (int j = 0; j < 4; ++j)
    if (base + j < n) s += count[base + j];
  long long total;
  block_excl_scan_256(s, s_wave, total);
  if (threadIdx.x == 0) part[blockIdx.x] = total;
}

__global__ void __launch_bounds__(256) k_scan_parts(long long* __restrict__ part, long long n_part) {
  __shared__ long long s_wave[4];
  __shared__ long long s_carry;
  if (threadIdx.x == 0) s_carry = 0;
  __syncthreads();
  for (long long b = 0; b < n_part; b += 256) {
    const long long i = b + threadIdx.x;
    const long long x = i < n_part ? part[i] : 0;
    long long total;
    const long long ex = block_excl_scan_256(x, s_wave, total);
    const long long carry = s_carry;
    if (i < n_part) part[i] = carry + ex;
    __syncthreads();
    if (threadIdx.x == 0) s_carry = carry + total;
    __syncthreads();
  }
}

__global__ void __launch_bounds__(256) k_scan_final(const int* __restrict__ count, long long n,
                                                    const long long* __restrict__ part, int* __restrict__ offs,
                                                    long long* __restrict__ total_out) {
  __shared__ long long s_wave[4];
  const long long base = (long long)blockIdx.x * 1024 + threadIdx.x * 4;
  int c[4];
  long long s = 0;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    c[j] = base + j < n ? count[base + j] : 0;
    s += c[j];
  }
  long long total;
  long long ex = block_excl_scan_256(s, s_wave, total) + part[blockIdx.x];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    if (base + j < n) offs[base + j] = sat_int(ex);
    ex += c[j];
    if (base + j == n - 1) {
      offs[n] = sat_int(ex);
      *total_out = ex;
    }
  }
}

// ----------------------------------------------------------------- fill
// Each workgroup counts its entries per tile in LDS, reserves one contiguous
// range per tabled tile with a single global atomic, then writes its entries:
// into that range, or for a tile the table did not take, at a position taken
// from the tile's global counter.  Both passes must agree on which entries
// are tabled (tile_slot without CUTOFF); then every tile's counter ends at 0
// and each position of its list is written once.
__global__ void __launch_bounds__(kBinBlock) k_fill(const mer_view* __restrict__ views, int n_views,
                                              const long long* __restrict__ tri_base,
                                              const long long* __restrict__ tile_base, long long total_tris,
                                              int tw_log2, int th_log2, int big_tiles, const Rec* __restrict__ rec,
                                              const BBox* __restrict__ bbox,
                                              int* __restrict__ count, const int* __restrict__ offs,
                                              long long bin_cap, int* __restrict__ bins) {
  __shared__ int s_tkey[kBinSlots], s_tcnt[kBinSlots], s_toff[kBinSlots], s_nocc;
  clear_tile_table(s_tkey, s_tcnt, &s_nocc);
  __syncthreads();
  const long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  BBox bb = {1, 1, 0, 0};
  if (g < total_tris) bb = bbox[g];
  const bool live = bb.x0 <= bb.x1 && box_tiles(bb, tw_log2, th_log2) <= big_tiles;  // large ones: k_bin_big
  Rec R;
  R.tl = 0;
  int W = 0;
  long long base = 0;
  // the count pass's masks when every triangle of the wave has one (one
  // walk for the whole wave), else the same tests again
  bool masked = false;
  auto each_tile = [&](auto f) {
    if (masked) for_each_masked_tile((unsigned)R.tl >> 16, bb, W, base, tw_log2, th_log2, f);
    else for_each_tile(R, bb, W, base, tw_log2, th_log2, f);
  };
  if (live) {
    const int vi = wave_bucket(tri_base, n_views, g);
    W = views[vi].W;
    base = tile_base[vi];
    R.tl = rec[g].tl;
  }
  masked = __ballot(live && !(R.tl & kMaskValid)) == 0ull;
  if (live && !masked) R = rec[g];  // the whole record only for the tests
  if (live) {
    each_tile([&](int gt) {
      const int sl = tile_slot<true, false>(s_tkey, &s_nocc, gt);
      if (sl >= 0) atomicAdd(&s_tcnt[sl], 1);
    });
  }
  __syncthreads();
  for (int i = threadIdx.x; i < kBinSlots; i += blockDim.x) {
    const int gt = s_tkey[i];
    if (gt >= 0) {
      const int n = s_tcnt[i];
      s_toff[i] = offs[gt];
      s_tcnt[i] = atomicSub(count + gt, n) - n;  // this workgroup's range within the tile
    }
  }
  __syncthreads();
  // the table is frozen: a tile in it takes the next position of the
  // workgroup's range, any other tile its own global counter
  if (live) {
    each_tile([&](int gt) {
      const int sl = tile_slot<false, false>(s_tkey, &s_nocc, gt);
      const long long pos = sl >= 0 ? (long long)s_toff[sl] + atomicAdd(&s_tcnt[sl], 1)
                                    : (long long)offs[gt] + (atomicSub(count + gt, 1) - 1);
      if (pos < bin_cap) bins[pos] = (int)g;
    });
  }
}

// ----------------------------------------------------- large triangles
// The count pass leaves one list of large triangles per workgroup.  The scan
// kernels turn the list lengths into offsets and a total, k_big_pack copies
// the lists into one flat list, and k_bin_big walks it: wave v takes
// triangles v, v + (waves), ... and covers each one's tiles with all 64
// lanes, straight into the tile counters (one large triangle's tiles are
// distinct).  FILL = false counts, true writes entries.
constexpr int kBigGrid = 2048;

__global__ void __launch_bounds__(kBinBlock) k_big_pack(const int* __restrict__ big, const int* __restrict__ big_n,
                                                        const int* __restrict__ big_off, int* __restrict__ flat) {
  const int n = big_n[blockIdx.x];
  if ((int)threadIdx.x < n)
    flat[big_off[blockIdx.x] + threadIdx.x] = big[(long long)blockIdx.x * kBinBlock + threadIdx.x];
}

template <bool FILL>
__global__ void __launch_bounds__(256) k_bin_big(const mer_view* __restrict__ views, int n_views,
                                                 const long long* __restrict__ tri_base,
                                                 const long long* __restrict__ tile_base, int tw_log2, int th_log2,
                                                 const Rec* __restrict__ rec, const BBox* __restrict__ bbox,
                                                 const int* __restrict__ flat, const long long* __restrict__ status,
                                                 int* __restrict__ count, const int* __restrict__ offs,
                                                 long long bin_cap, int* __restrict__ bins) {
  const long long n_big = status[4];
  const long long waves = (long long)gridDim.x * (blockDim.x >> 6);
  for (long long i = (long long)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); i < n_big; i += waves) {
    const long long g = __builtin_amdgcn_readfirstlane(flat[i]);
    const int vi = __builtin_amdgcn_readfirstlane(find_bucket(tri_base, n_views, g));
    const BBox bb = bbox[g];
    const Rec R = rec[g];
    wave_each_tile(R, bb, views[vi].W, tile_base[vi], tw_log2, th_log2, [&](int gt) {
      if (FILL) {
        const long long pos = (long long)offs[gt] + (atomicSub(count + gt, 1) - 1);
        if (pos < bin_cap) bins[pos] = (int)g;
      } else {
        atomicAdd(count + gt, 1);
      }
    });
  }
}

// --------------------------------------------------------------- raster
// Per (record, tile) constants, prepared by one lane per record and read by
// every lane of the tile from LDS (same address in every lane: broadcast).
// A record is "fast" when |A|, |B| < 2^17 (pixel offsets from the tile origin
// fit in 31 bits) and |D| < 2^31: a covered centre's unbiased edge values lie
// in [0, |D|], so they are the 32-bit sum of the tile-origin values' low
// halves and the offsets, and d = |D| is the same at every pixel.  A fast
// record's vertex 1/z also lie in [2^-64, 2^64], which keeps every step of
// div_rn below a normal number.
struct __align__(16) TileRec {
  int A[3];
  int B[3];
  int u0[3];   // low 32 bits of the unbiased edge values at the tile origin
  int thr[3];  // covered iff offset_k > thr_k (minus the biased value, clamped)
  float q[3];  // vertex 1/z
  float d;     // (float)|D|
  float qb;    // early-z bound: no key of this record exceeds it
  unsigned tneg;  // ~t (t the triangle index in the view), low half of the visibility key; 0: skip
  float rd;    // RN(1 / d)
  int fast;
};
static_assert(sizeof(TileRec) == 80, "tile record layout");

// RN(a / b) from y = RN(1 / b), for a >= 0 and b >= 1 with every step a
// normal number: q0 = RN(a y) is within 1.5 ulp of a / b, one correction
// with the remainder (exact product in the fma) brings it within one ulp,
// and then the remainder is exact and one more correction gives the
// correctly rounded quotient (Markstein's theorem on division with a fused
// multiply-add).  Five operations in place of the division's scale, fix-up
// and reciprocal sequence; the result is the IEEE quotient bit for bit.
__device__ __forceinline__ float div_rn(float a, float b, float y) {
  const float q0 = a * y;
  const float q1 = fmaf(fmaf(-b, q0, a), y, q0);
  return fmaf(fmaf(-b, q1, a), y, q1);
}

// TRACK: keep the winner's barycentrics along the candidate loop, formed
// from its depth-key products with the resolve's own arithmetic (for stored
// barycentrics); without it the resolve recomputes them from the winner's
// vertices when it interpolates.  bary (TRACK only) and out may be NULL.
template <int TW, int TH, bool TRACK>
__global__ void __launch_bounds__(TW* TH) __attribute__((amdgpu_waves_per_eu(8))) k_raster(const mer_view* __restrict__ views, int n_views,
                                                   const long long* __restrict__ tri_base,
                                                   const long long* __restrict__ tile_base,
                                                   const Rec* __restrict__ rec, const BBox* __restrict__ bbox,
                                                   const int* __restrict__ offs, const int* __restrict__ bins,
                                                   const int* __restrict__ count,
                                                   long long bin_cap, const unsigned long long* __restrict__ key,
                                                   long long px_begin, const float* __restrict__ v,
                                                   const int32_t* __restrict__ tri, int32_t* __restrict__ tri_id,
                                                   float* __restrict__ depth, float* __restrict__ bary,
                                                   long long* __restrict__ status, const float* __restrict__ attr,
                                                   int C_a, int append_z, float* __restrict__ out) {
  constexpr int NT = TW * TH;
  __shared__ TileRec s_tr[NT];
  // single-wave tiles: the chunk's records go to s_tr nearest first.  The
  // sort keys share the first bytes of s_tr: the wave reads every key before
  // any lane stores its record (LDS operations of one wave complete in
  // order), and the keys are dead by then.
  constexpr bool kSort = NT == 64;
  unsigned* const s_ks = reinterpret_cast<unsigned*>(s_tr);
  const long long g = xcd_tile(blockIdx.x, gridDim.x);
  const int lt = threadIdx.x;
  const int vi = __builtin_amdgcn_readfirstlane(find_bucket(tile_base, n_views, g));
  const mer_view vw = views[vi];
  const long long local = g - tile_base[vi];
  const int tiles_x = (vw.W + TW - 1) / TW;
  int x0, y0;
  grid_xy(local, tiles_x, x0, y0);
  x0 *= TW;
  y0 *= TH;
  const int lx = lt % TW, ly = lt / TW;
  const int px = x0 + lx, py = y0 + ly;
  const int dxs = lx * 256, dys = ly * 256;
  const bool inside = px < vw.W && py < vw.H;
  const long long tb = tri_base[vi], tb_end = tri_base[vi + 1];

  const long long start = offs[g], end = offs[g + 1];
  const bool overflow = end > bin_cap;
  // overflow fallback: scan every record of the view, filtered by bbox
  const long long n_items = overflow ? (tb_end - tb) : (end - start);
  if (lt == 0) {
    if (overflow) atomicAdd((unsigned long long*)status, 1ull);
    // integrity: the fill passes take every tile counter back to 0
    if (count[g] != 0) atomicAdd((unsigned long long*)status + 6, 1ull);
  }

  // key: the small-triangle pass's result, or NULL when that pass is off
  unsigned long long best = inside && key ? key[vw.px_off - px_begin + (long long)py * vw.W + px] : 0ull;
  // the current winner's barycentrics when it came from this loop, from its
  // products e_k q_k with the resolve's arithmetic: no gather afterwards
  float wb0 = 0.f, wb1 = 0.f;
  bool own = false;
  const unsigned long long inside_m = __builtin_amdgcn_ballot_w64(inside);
  for (long long c0 = 0; c0 < n_items; c0 += NT) {
    const int n = (int)min((long long)NT, n_items - c0);
    bool is_fast = false, is_slow = false;
    if (lt < n) {
      long long r;
      bool keep = true;
      if (!overflow) {
        r = bins[start + c0 + lt];
        // integrity: a bin entry names a record of this tile's view; any
        // other value is counted (mer_status fails on it) and not read
        if (r < tb || r >= tb_end) {
          keep = false;
          atomicAdd((unsigned long long*)status + 5, 1ull);
        }
      } else {
        r = tb + c0 + lt;
        const BBox bb = bbox[r];
        keep = bb.x0 <= bb.x1 && bb.x1 >= x0 && bb.x0 < x0 + TW && bb.y1 >= y0 && bb.y0 < y0 + TH;
      }
      TileRec o;
      o.tneg = 0u;
      o.fast = 0;
      if (keep) {
        const Rec R = rec[r];
        long long Dabs = 0;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          // exact biased edge value at the tile origin's centre
          const long long Et = (long long)R.A[k] * (long long)(x0 * 256) + (long long)R.B[k] * (long long)(y0 * 256) + R.C[k];
          const long long u = Et - ((R.tl >> k) & 1);
          Dabs += u;  // the unbiased values sum to |D| at every point
          const long long nt = -Et;
          o.thr[k] = nt > 2147483647ll ? 2147483647 : (nt < -2147483647ll ? -2147483647 : (int)nt);
          o.u0[k] = (int)(unsigned)(unsigned long long)u;
          o.A[k] = R.A[k];
          o.B[k] = R.B[k];
          o.q[k] = R.q[k];
        }
        o.d = (float)Dabs;
        o.rd = 1.0f / o.d;
        const float qlo = fminf(R.q[0], fminf(R.q[1], R.q[2])), qhi = fmaxf(R.q[0], fmaxf(R.q[1], R.q[2]));
        o.fast = (R.tl & 8) && Dabs < 2147483648ll && qlo >= 0x1p-64f && qhi <= 0x1p64f;
        // Early z: the key is a convex combination of the vertices' 1/z up to
        // a few roundings (< 2^-20 relative), so a lane whose surface is
        // already strictly nearer than every vertex skips the key (it could
        // not win, not even the tie on equal 1/z).  The test is per lane, so
        // it holds for every tile shape.  The bound is rounded up to the top
        // of its group of 64 floats (still a bound, and at least the smallest
        // normal): the sort key below keeps only the group, and the bound
        // must not increase along the sorted order.
        const unsigned qbits = __float_as_uint(fmaxf(qhi * (1.0f + 0x1p-20f), 0x1p-126f));
        o.qb = __uint_as_float(qbits < 0x7F800000u ? qbits | 63u : qbits);
        o.tneg = ~(unsigned)(r - tb);
        is_fast = o.fast;
        is_slow = !o.fast;
      }
      if constexpr (kSort)
        s_ks[lt] = (is_fast ? __float_as_uint(o.qb) & ~63u : is_slow ? 64u : 0u) | (unsigned)(63 - lt);
      else s_tr[lt] = o;
      if constexpr (kSort) {
        // The winner is the largest key whatever the order, so the chunk is
        // taken nearest first: record i goes to its rank by sort key, which
        // puts the fast records first, by early-z bound (descending), then
        // the slow ones, then the skipped ones.  The key's low six bits hold
        // 63 - i, so keys are distinct and the ranks a permutation.  Once no
        // lane's surface is as far as a fast record's bound, no later fast
        // record can win.
        __builtin_amdgcn_wave_barrier();
        const unsigned mk = s_ks[lt];
        int rank = 0;
        for (int i = 0; i < n; ++i) rank += s_ks[i] > mk;
        s_tr[rank] = o;
      }
    }
    // single-wave tiles: fast records at ranks [0, n_fast), slow ones next
    const int n_fast = kSort ? (int)__popcll(__builtin_amdgcn_ballot_w64(is_fast)) : 0;
    const int n_slow = kSort ? (int)__popcll(__builtin_amdgcn_ballot_w64(is_slow)) : 0;
    __syncthreads();
    // Fast records here; the others (rare: long edges or a large |D|) after
    // the loop, so that this loop carries the winner through one path only.
    // The break leaves out only fast records that cannot win (their bound
    // is below every lane's key); the second loop tests every slow record.
    bool slow = false;
    for (int j = 0; j < (kSort ? n_fast : n); ++j) {
      // the bound first, the rest of the record once it is taken (LDS
      // broadcasts: every lane reads the same address)
      const float qb = s_tr[j].qb, rd = s_tr[j].rd;
      const unsigned tneg = s_tr[j].tneg;
      if (!kSort && !tneg) continue;  // uniform across the block
      const float best_q = key_q(best);
      const unsigned long long near_m = __builtin_amdgcn_ballot_w64(qb >= best_q) & inside_m;
      if (kSort && !near_m) break;  // nor can any fast record after it
      if (!kSort && !s_tr[j].fast) {
        slow = true;
        continue;
      }
      const TileRec& T = s_tr[j];
      // covered iff off_k > thr_k for all k; then the unbiased edge values
      // are u0_k + off_k exactly (mod 2^32 and in [0, 2^31))
      int off[3];
      bool cov = inside & (qb >= best_q);
      unsigned long long cov_m = near_m;
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        off[k] = __mul24(T.A[k], dxs) + __mul24(T.B[k], dys);  // 24-bit signed products
        cov &= off[k] > T.thr[k];
        cov_m &= __builtin_amdgcn_ballot_w64(off[k] > T.thr[k]);
      }
      // taken by the whole wave when any lane is covered (a wave-uniform
      // branch): uncovered lanes compute values they never keep
      if (cov_m) {
        float e[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) e[i] = (float)(int)((unsigned)T.u0[i] + (unsigned)off[i]);
        const float a = e[0] * T.q[0];
        const float b = e[1] * T.q[1];
        const float c = e[2] * T.q[2];
        float nq = a + b;
        nq = nq + c;
        const float qk = div_rn(nq, T.d, rd);  // == nq / T.d where covered
        const unsigned long long k = ((unsigned long long)__float_as_uint(qk) << 32) | tneg;
        const bool win = cov && k > best;
        best = win ? k : best;
        if (TRACK) {
          const float r = __builtin_amdgcn_rcpf(nq);
          const float x0 = a * r, x1 = b * r;
          wb0 = win ? x0 : wb0;
          wb1 = win ? x1 : wb1;
          own |= win;
        }
      }
    }
    if (kSort ? n_slow > 0 : slow) {
      for (int j = kSort ? n_fast : 0; j < (kSort ? n_fast + n_slow : n); ++j) {
        const TileRec T = s_tr[j];
        if (!kSort && (!T.tneg || T.fast)) continue;
        const int t = (int)~T.tneg;
        const Rec R = rec[tb + __builtin_amdgcn_readfirstlane(t)];
        long long E[3];
#pragma unroll
        for (int k = 0; k < 3; ++k)
          E[k] = (long long)R.A[k] * (long long)(px * 256) + (long long)R.B[k] * (long long)(py * 256) + R.C[k];
        if (inside && covered(E) && T.qb >= key_q(best)) {
          float e[3], d;
          edge_values(R, E, e, d);
          const float a = e[0] * R.q[0];
          const float b = e[1] * R.q[1];
          const float c = e[2] * R.q[2];
          float nq = a + b;
          nq = nq + c;
          const unsigned long long k = vis_key(nq / d, t);
          const bool win = k > best;
          best = win ? k : best;
          if (TRACK) {
            const float r = __builtin_amdgcn_rcpf(nq);
            const float x0 = a * r, x1 = b * r;
            wb0 = win ? x0 : wb0;
            wb1 = win ? x1 : wb1;
            own |= win;
          }
        }
      }
    }
    __syncthreads();
  }
  if (!inside) return;
  // the pixel's index from the pixel coordinates again here: a 64-bit value
  // kept across the loop would cost registers the loop needs
  int pxr = px, pyr = py;
  asm volatile("" : "+v"(pxr), "+v"(pyr));
  const long long p = vw.px_off + (long long)pyr * vw.W + pxr;
  const int t = key_tri(best);
  tri_id[p] = t;
  if (depth) depth[p] = t >= 0 ? 1.0f / key_q(best) : 0.0f;
  if (TRACK || out) {
    float b0 = 0.f, b1 = 0.f;
    if (t >= 0) {
      // a winner not tracked here (small-triangle pass, or no tracking): the
      // same products from its vertices
      if (TRACK && own) {
        b0 = wb0;
        b1 = wb1;
      } else {
        float wa, wb, wn;
        resolve_products(snap_triangle(v, vw, tri_row(tri, vw, t)), px, py, wa, wb, wn);
        const float r = __builtin_amdgcn_rcpf(wn);
        b0 = wa * r;
        b1 = wb * r;
      }
    }
    if (TRACK && bary) {
      bary[2 * p] = b0;
      bary[2 * p + 1] = b1;
    }
    if (out) {
      // interpolation, with the arithmetic of the interpolation kernel, four
      // channels a load and a store where the channel counts allow
      const int C = C_a + append_z;
      float* o = out + p * C;
      const int vout = row_vec(C, out);
      const bool a_al = ((vw.a_off * C_a) & 3) == 0;
      const int va = row_vec(C_a, attr) == 3 ? 3 : row_vec(C_a, attr) == 4 && a_al ? 4 : 0;
      float b2 = 0.f, zv = 0.f;
      const float *a0 = attr, *a1 = attr, *a2 = attr;
      if (t >= 0) {
        b2 = (1.0f - b0) - b1;
        const int32_t* row = tri_row(tri, vw, t);
        const int i0 = row[0], i1 = row[1], i2 = row[2];
        a0 = attr + (vw.a_off + i0) * C_a;
        a1 = attr + (vw.a_off + i1) * C_a;
        a2 = attr + (vw.a_off + i2) * C_a;
        if (append_z) {
          const float* vb = v + vw.v_off * 3;
          const float z0 = vb[(size_t)i0 * 3 + 2], z1 = vb[(size_t)i1 * 3 + 2], z2 = vb[(size_t)i2 * 3 + 2];
          zv = (b0 * z0 + b1 * z1) + b2 * z2;
        }
      }
      for (int c0 = 0; c0 < C; c0 += 4) {
        const int n = min(4, C - c0);
        float xs[4] = {0.f, 0.f, 0.f, 0.f};
        if (t >= 0) {
          if (c0 < C_a) {
            const int na = min(4, C_a - c0);
            const float4 x0 = row4(a0 + c0, va, na), x1 = row4(a1 + c0, va, na), x2 = row4(a2 + c0, va, na);
#pragma unroll
            for (int j = 0; j < 4; ++j)
              if (j < na) xs[j] = (b0 * f4(x0, j) + b1 * f4(x1, j)) + b2 * f4(x2, j);
          }
#pragma unroll
          for (int j = 0; j < 4; ++j)
            if (append_z && c0 + j == C_a) xs[j] = zv;
        }
        if (vout == 4) {
          *reinterpret_cast<float4*>(o + c0) = make_float4(xs[0], xs[1], xs[2], xs[3]);
        } else if (vout == 3) {
          *reinterpret_cast<float3*>(o + c0) = make_float3(xs[0], xs[1], xs[2]);
        } else {
#pragma unroll
          for (int j = 0; j < 4; ++j)
            if (j < n) o[c0 + j] = xs[j];
        }
      }
    }
  }
}

// --------------------------------------------------------------- launch
int launch_rasterize(const mer_plan* P, const mer_view* views, const float* v, const int32_t* tri, int32_t* tri_id,
                     float* depth, float* bary, const float* attr, int C_a, int append_z, float* out, void* ws,
                     hipStream_t st) {
  char* w = (char*)ws;
  long long* viewtab = (long long*)(w + P->off_viewtab);
  long long* tri_base = viewtab;
  long long* tile_base = viewtab + (P->n_views + 1);
  Rec* rec = (Rec*)(w + P->off_rec);
  BBox* bbox = (BBox*)(w + P->off_bbox);
  int* count = (int*)(w + P->off_count);
  int* offs = (int*)(w + P->off_offs);
  long long* part = (long long*)(w + P->off_part);
  int* bins = (int*)(w + P->off_bins);
  long long* status = (long long*)(w + P->off_status);
  int* big = (int*)(w + P->off_big);
  int* big_n = (int*)(w + P->off_bign);
  int* big_off = big_n + P->n_bingroups;  // n_bingroups + 1 entries
  long long* big_part = (long long*)(w + P->off_bigpart);
  int* big_flat = (int*)(w + P->off_bigflat);
  unsigned long long* key = (unsigned long long*)(w + P->off_key);
  const long long npx = P->total_px - P->px_begin;
  const int twl = __builtin_ctz(P->tile_w), thl = __builtin_ctz(P->tile_h);

  hipLaunchKernelGGL(k_prep, dim3(1), dim3(1024), 0, st, views, P->n_views, twl, thl, tri_base, tile_base, status);
  const long long nt = P->total_tiles;
  hipLaunchKernelGGL(k_zero_i32, dim3((unsigned)min((nt + 255) / 256, 4096ll)), dim3(256), 0, st, count, nt);
  if (P->small_px > 0)
    hipLaunchKernelGGL(k_zero_u64, dim3((unsigned)min((npx + 255) / 256, 8192ll)), dim3(256), 0, st, key, npx);
  else
    key = nullptr;  // no small-triangle pass: every pixel starts from background
  if (P->total_tris > 0) {
    const dim3 bgrid((unsigned)((P->total_tris + kBinBlock - 1) / kBinBlock)), bblock(kBinBlock);
    hipLaunchKernelGGL(k_setup, bgrid, bblock, 0, st, views, P->n_views, v, tri, tri_base, tile_base, P->total_tris,
                       twl, thl, P->small_px, (int)P->big_tiles, P->px_begin, rec, bbox, count, key, status, big,
                       big_n);
    const long long nl = bgrid.x, nlp = (nl + 1023) / 1024;  // list lengths -> offsets, total in status[4]
    hipLaunchKernelGGL(k_scan_partial, dim3((unsigned)nlp), dim3(256), 0, st, big_n, nl, big_part);
    hipLaunchKernelGGL(k_scan_parts, dim3(1), dim3(256), 0, st, big_part, nlp);
    hipLaunchKernelGGL(k_scan_final, dim3((unsigned)nlp), dim3(256), 0, st, big_n, nl, big_part, big_off, status + 4);
    hipLaunchKernelGGL(k_big_pack, bgrid, bblock, 0, st, big, big_n, big_off, big_flat);
    hipLaunchKernelGGL(k_bin_big<false>, dim3(kBigGrid), dim3(256), 0, st, views, P->n_views, tri_base, tile_base, twl,
                       thl, rec, bbox, big_flat, status, count, offs, P->bin_cap, bins);
  }
  hipLaunchKernelGGL(k_scan_partial, dim3((unsigned)P->n_part), dim3(256), 0, st, count, nt, part);
  hipLaunchKernelGGL(k_scan_parts, dim3(1), dim3(256), 0, st, part, P->n_part);
  hipLaunchKernelGGL(k_scan_final, dim3((unsigned)P->n_part), dim3(256), 0, st, count, nt, part, offs, status + 2);
  if (P->total_tris > 0) {
    const dim3 bgrid((unsigned)((P->total_tris + kBinBlock - 1) / kBinBlock)), bblock(kBinBlock);
    hipLaunchKernelGGL(k_fill, bgrid, bblock, 0, st, views, P->n_views, tri_base, tile_base, P->total_tris, twl, thl,
                       (int)P->big_tiles, rec, bbox, count, offs, P->bin_cap, bins);
    hipLaunchKernelGGL(k_bin_big<true>, dim3(kBigGrid), dim3(256), 0, st, views, P->n_views, tri_base, tile_base, twl,
                       thl, rec, bbox, big_flat, status, count, offs, P->bin_cap, bins);
  }
#define MER_RASTER(TW, TH)                                                                               \
  do {                                                                                                   \
    if (bary)                                                                                            \
      hipLaunchKernelGGL((k_raster<TW, TH, true>), dim3((unsigned)nt), dim3(TW * TH), 0, st, views,      \
                         P->n_views, tri_base, tile_base, rec, bbox, offs, bins, count, P->bin_cap, key, \
                         P->px_begin, v, tri, tri_id, depth, bary, status, attr, C_a, append_z, out);    \
    else                                                                                                 \
      hipLaunchKernelGGL((k_raster<TW, TH, false>), dim3((unsigned)nt), dim3(TW * TH), 0, st, views,     \
                         P->n_views, tri_base, tile_base, rec, bbox, offs, bins, count, P->bin_cap, key, \
                         P->px_begin, v, tri, tri_id, depth, bary, status, attr, C_a, append_z, out);    \
  } while (0)
  if (P->tile_w == 8 && P->tile_h == 8) MER_RASTER(8, 8);
  else if (P->tile_w == 16 && P->tile_h == 16) MER_RASTER(16, 16);
  else if (P->tile_w == 32 && P->tile_h == 8) MER_RASTER(32, 8);
  else if (P->tile_w == 16 && P->tile_h == 8) MER_RASTER(16, 8);
  else return MER_ETUNING;
#undef MER_RASTER
  return hipGetLastError() == hipSuccess ? MER_OK : MER_ELAUNCH;
}

}  // namespace mer
