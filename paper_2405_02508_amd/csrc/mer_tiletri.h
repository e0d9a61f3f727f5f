// mer_tiletri.h -- the distinct triangles seen by a square pixel tile and its
// one-pixel border, snapped once each into LDS.
//
// A per-pixel sweep that visits every pixel's triangle and the triangles of
// its four neighbours would otherwise re-load and re-snap the same triangle
// many times, each time through a chain of dependent loads (index image ->
// index row -> vertices).  Here the workgroup collects the ids of its tile's
// pixels and of the border pixels, de-duplicates them in an LDS hash
// table, and snaps each distinct triangle once, all lanes in parallel; later
// per-pixel steps read the snapped triangles from LDS.
#pragma once
#include "mer_device.h"

namespace mer {

// TS: tile side in pixels (8 or 16); the workgroup has TS * TS threads.
template <int TS>
struct TileDims {
  static constexpr int G = TS + 2;              // grid side with the border
  static constexpr int Cap = TS * TS + 4 * TS;  // distinct ids at most: tile + border (no corners)
  static constexpr int Hash = TS == 16 ? 512 : 128;  // hash slots (power of two, > Cap)
  static constexpr int HashBits = TS == 16 ? 9 : 7;
};

// DV: also stage the three vertices' tangent rows (9 floats) per triangle.
// Records hold the snapped coordinates, vertex indices (idx[0] = -1 for a
// triangle that does not snap) and z; 1/z and twice the area are recomputed
// on reading (bit-identical to the snap's own values).
template <int TS, bool DV>
struct TileTris {
  using Dm = TileDims<TS>;
  int key[Dm::Hash];        // hash keys (triangle id), -1 empty
  int dense[Dm::Hash];      // record index of each occupied slot
  int grid[Dm::G * Dm::G];  // hash slot per grid position, -1 background / outside
  int n;                    // distinct triangles
  int X[3][Dm::Cap], Y[3][Dm::Cap], idx[3][Dm::Cap];
  int zb[3][Dm::Cap];       // bits of z; zb[2] holds the record's triangle id until it is snapped
  float dv[DV ? 9 : 1][DV ? Dm::Cap : 1];
};

template <int TS>
__device__ __forceinline__ int tt_pos(int lx, int ly) { return (ly + 1) * TileDims<TS>::G + (lx + 1); }

// All TS * TS threads of the workgroup call this.  Tile origin (x0, y0) of
// view vw; thread i owns pixel (x0 + i % TS, y0 + i / TS), threads
// 0 .. 4 TS - 1 also one border pixel each.  On return (after a barrier) the grid and the
// records are valid (read them with tile_rec).  dv may be NULL (then the
// tangent rows are not set).
template <int TS, bool DV>
__device__ void tile_tris_build(TileTris<TS, DV>& T, const mer_view& vw, int x0, int y0,
                                const int32_t* __restrict__ tri_id, const int32_t* __restrict__ tri,
                                const float* __restrict__ v, const float* __restrict__ dv) {
  using Dm = TileDims<TS>;
  const int i = threadIdx.x;
  for (int s = i; s < Dm::Hash; s += TS * TS) T.key[s] = -1;
  if (i == 0) T.n = 0;
  // the two positions this thread reads: its pixel and (i < 4 TS) a border pixel
  int lx[2], ly[2], id[2] = {-1, -1};
  lx[0] = i % TS;
  ly[0] = i / TS;
  const int side = i / TS, j = i % TS;  // for i < 4 TS: top, bottom, left, right
  lx[1] = side == 0 || side == 1 ? j : side == 2 ? -1 : TS;
  ly[1] = side == 0 ? -1 : side == 1 ? TS : j;
#pragma unroll
  for (int r = 0; r < 2; ++r) {
    if (r == 1 && i >= 4 * TS) break;
    const int x = x0 + lx[r], y = y0 + ly[r];
    if (x < 0 || y < 0 || x >= vw.W || y >= vw.H) continue;
    int t = tri_id[vw.px_off + (long long)y * vw.W + x];
    id[r] = (t >= 0 && t < vw.n_t) ? t : -1;
  }
  __syncthreads();  // key[] cleared
  // a triangle meets a row of pixels in one run (it is convex): only the
  // first pixel of each run inserts, the others take its slot
  const int lane = i & 63;
  const int id_prev = __shfl_up(id[0], 1, 64);
  const bool head = i % TS == 0 || id[0] != id_prev;
#pragma unroll
  for (int r = 0; r < 2; ++r) {
    int slot = -1;
    if (id[r] >= 0 && (r == 1 || head)) {
      unsigned h = ((unsigned)id[r] * 2654435761u) >> (32 - Dm::HashBits);
      // at most Cap < Hash distinct keys: a free or matching slot exists
      for (;;) {
        const int s = (int)(h & (Dm::Hash - 1));
        const int old = atomicCAS(&T.key[s], -1, id[r]);
        if (old == -1 || old == id[r]) {
          slot = s;
          break;
        }
        ++h;
      }
    }
    if (r == 0) {
      const unsigned long long F = __ballot(head);
      const unsigned long long upto = lane == 63 ? ~0ull : ((2ull << lane) - 1ull);
      const int hl = 63 - __clzll((long long)(F & upto));
      slot = __shfl(slot, hl, 64);
    } else if (i >= 4 * TS) {
      break;
    }
    T.grid[tt_pos<TS>(lx[r], ly[r])] = slot;
  }
  if (i < 4) T.grid[(i >> 1) * (Dm::G - 1) * Dm::G + (i & 1) * (Dm::G - 1)] = -1;  // corners (never read)
  __syncthreads();  // keys final
  // record indices: one atomic per wave, lanes ranked by a ballot
  for (int s = i; s < Dm::Hash; s += TS * TS) {
    const int k = T.key[s];
    const unsigned long long M = __ballot(k >= 0);
    int base = 0;
    if (lane == 0 && M) base = atomicAdd(&T.n, (int)__popcll(M));
    base = __shfl(base, 0, 64);
    if (k < 0) continue;
    const int d = base + (int)__popcll(M & ((1ull << lane) - 1ull));
    T.dense[s] = d;
    T.zb[2][d] = k;
  }
  __syncthreads();  // record indices final
  // one record per distinct triangle, snapped once
  const int n = T.n;
  for (int d = i; d < n; d += TS * TS) {
    const int32_t* row = tri_row(tri, vw, T.zb[2][d]);
    int vid[3];
    bool iok = true;
#pragma unroll
    for (int m = 0; m < 3; ++m) {
      vid[m] = row[m];
      iok &= (unsigned)vid[m] < (unsigned)vw.n_v;
    }
    float dd[9];
    if constexpr (DV) {
      // the tangent rows load with the vertices (same indices, same step)
      if (iok && dv) {
#pragma unroll
        for (int m = 0; m < 3; ++m) {
          const float* r = dv + (vw.v_off + vid[m]) * 3;
          dd[3 * m] = r[0];
          dd[3 * m + 1] = r[1];
          dd[3 * m + 2] = r[2];
        }
      }
    }
    const Snap sn = snap_triangle<false>(v, vw, row);
#pragma unroll
    for (int m = 0; m < 3; ++m) {
      T.X[m][d] = sn.X[m];
      T.Y[m][d] = sn.Y[m];
      T.idx[m][d] = sn.ok ? sn.idx[m] : -1;
      T.zb[m][d] = __float_as_int(sn.z[m]);
    }
    if constexpr (DV) {
      if (iok && dv) {
#pragma unroll
        for (int m = 0; m < 9; ++m) T.dv[m][d] = dd[m];
      }
    }
  }
  __syncthreads();  // records written
}

// Record index at grid position (lx, ly) in [-1, TS]^2, or -1 for
// background, outside the view, or a triangle that does not snap.
template <int TS, bool DV>
__device__ __forceinline__ int tile_rec(const TileTris<TS, DV>& T, int lx, int ly) {
  const int s = T.grid[tt_pos<TS>(lx, ly)];
  if (s < 0) return -1;
  const int d = T.dense[s];
  return T.idx[0][d] >= 0 ? d : -1;
}

// Snapped triangle of record d (d >= 0), as snap_triangle<false> gives it.
template <int TS, bool DV>
__device__ __forceinline__ Snap tile_snap(const TileTris<TS, DV>& T, int d) {
  Snap s;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    s.X[k] = T.X[k][d];
    s.Y[k] = T.Y[k][d];
    s.idx[k] = T.idx[k][d];
    s.z[k] = __int_as_float(T.zb[k][d]);
    s.q[k] = __builtin_amdgcn_rcpf(s.z[k]);
  }
  s.D = (long long)(s.X[1] - s.X[0]) * (long long)(s.Y[2] - s.Y[0]) -
        (long long)(s.X[2] - s.X[0]) * (long long)(s.Y[1] - s.Y[0]);
  s.ok = true;
  return s;
}

}  // namespace mer
