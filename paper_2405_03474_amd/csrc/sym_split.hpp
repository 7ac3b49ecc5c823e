// Index arithmetic of the symmetric split of an on-the-fly product (M is
// symmetric, Section 2): M is cut into 128 x 128 blocks and only the blocks
// on and above the diagonal are generated; block (I, J), J > I, feeds rows I
// directly and rows J transposed.
//
// Units: the column blocks are grouped into strips of `ms` blocks; unit
// (S, I) is row tile I of strip S, i.e. the blocks J >= I of the strip, for
// I = 0 .. me(S) - 1 with me(S) = min(ms (S + 1), nblk).  Units are numbered
// strip-major.  A unit costs one step per block; workgroup g takes the units
// u whose cost before u, times G, lies in [g cost, (g + 1) cost).
//
// Partial sums (tiles of 128 rows x the product's columns): one direct slot
// per unit, grouped by row tile (row tile R's slots, for strips R / ms ..
// ns - 1, are contiguous, so its epilogue streams one range), then, per
// workgroup, ms transposed slots (one per block of the strip) for each strip
// it touches, at index units + (g Jt + S - first strip of g) ms + (J - ms S).
// Row tile R's output is its direct slots in strip order followed by the
// transposed slots of the workgroups that own units (R / ms, I < R), in that
// order.
//
// Header-only and free of HIP types, so that host code (and a host-compiled
// check of the partition) uses the same functions as the kernels.
#pragma once

#include <cmath>
#include <cstdint>

#if !defined(__HIPCC__)
#ifndef __host__
#define __host__
#endif
#ifndef __device__
#define __device__
#endif
#endif

namespace ld {

struct SY {
  int64_t n, s, ld;
  int nblk;       // blocks per side (ceil(n / 128))
  int ms;         // blocks per strip
  int ns;         // strips
  int G;          // workgroups
  int Jt;         // transposed slot groups per workgroup (most strips one touches)
  int64_t units;  // (strip, row tile) units
  int64_t cost;   // blocks on or above the diagonal
};

__host__ __device__ inline int64_t sy_tri(int64_t x) { return x * (x + 1) / 2; }

// first unit of strip S (the strips before it have ms (S' + 1) row tiles)
__host__ __device__ inline int64_t sy_u0(const SY& p, int64_t S) { return p.ms * sy_tri(S); }

// rows tiles of strip S (one past its last column block)
__host__ __device__ inline int sy_me(const SY& p, int S) {
  return p.ms * (S + 1) < p.nblk ? p.ms * (S + 1) : p.nblk;
}

__host__ __device__ inline int sy_strip(const SY& p, int64_t u) {
  int64_t S = (int64_t)((sqrt(8.0 * (double)u / p.ms + 1.0) - 1.0) * 0.5);
  if (S > p.ns - 1) S = p.ns - 1;
  if (S < 0) S = 0;
  while (S > 0 && sy_u0(p, S) > u) --S;
  while (S + 1 < p.ns && sy_u0(p, S + 1) <= u) ++S;
  return (int)S;
}

// blocks in the units before unit u
__host__ __device__ inline int64_t sy_cost_before(const SY& p, int64_t u) {
  if (u >= p.units) return p.cost;
  const int64_t S = sy_strip(p, u);
  const int64_t I = u - sy_u0(p, S);
  const int64_t mS = p.ms * S;
  const int64_t meff = sy_me(p, (int)S) - mS;
  // row tiles 0 .. mS meet the whole strip, row tile mS + j meets meff - j blocks
  int64_t c = sy_tri(mS) + meff * (I < mS + 1 ? I : mS + 1);
  if (I > mS + 1) {
    const int64_t k = I - 1 - mS;
    c += k * meff - sy_tri(k);
  }
  return c;
}

// the workgroup of unit u, and the first unit of workgroup g (G: none left)
__host__ __device__ inline int sy_wg(const SY& p, int64_t u) {
  return (int)(sy_cost_before(p, u) * p.G / p.cost);
}
__host__ __device__ inline int64_t sy_start(const SY& p, int g) {
  if (g <= 0) return 0;
  if (g >= p.G) return p.units;
  const int64_t target = (int64_t)g * p.cost;
  int64_t lo = 0, hi = p.units;
  while (lo < hi) {
    const int64_t mid = (lo + hi) / 2;
    if (sy_cost_before(p, mid) * p.G >= target)
      hi = mid;
    else
      lo = mid + 1;
  }
  return lo;
}

// slot indices (in tiles): first direct slot of row tile R (the row tiles
// before it have ns - R' / ms slots each); direct slot of unit (S, I);
// transposed slot of column block J for workgroup g whose first strip is Sf,
// in strip S
__host__ __device__ inline int64_t sy_dir_base(const SY& p, int64_t R) {
  const int64_t q = R / p.ms, r = R % p.ms;
  return R * p.ns - (p.ms * (q * (q - 1) / 2) + q * r);
}
__host__ __device__ inline int64_t sy_dir_slot(const SY& p, int S, int I) {
  return sy_dir_base(p, I) + (S - I / p.ms);
}
__host__ __device__ inline int64_t sy_tr_slot(const SY& p, int g, int Sf, int S, int J) {
  return p.units + ((int64_t)g * p.Jt + (S - Sf)) * p.ms + (J - p.ms * S);
}

// the transposed slots of row tile R, in order; returns their count (at
// most cap are written)
__host__ __device__ inline int sy_tr_list(const SY& p, int R, int64_t* out, int cap) {
  const int SR = R / p.ms;
  const int64_t ub = sy_u0(p, SR) + R;
  int cnt = 0;
  int64_t u = sy_u0(p, SR);
  while (u < ub) {
    const int g = sy_wg(p, u);
    const int Sf = sy_strip(p, sy_start(p, g));
    if (cnt < cap) out[cnt] = sy_tr_slot(p, g, Sf, SR, R);
    ++cnt;
    u = sy_start(p, g + 1);
  }
  return cnt;
}

// the split of an n x s product over at most gmax workgroups (each with at
// least 4 ms blocks); Jt from the ranges.  Host-side.
inline SY sy_plan(int64_t n, int64_t s, int ms, int gmax) {
  SY p{};
  p.n = n;
  p.s = s;
  p.ld = s;
  p.nblk = (int)((n + 127) / 128);
  p.ms = ms;
  p.ns = (p.nblk + ms - 1) / ms;
  p.units = sy_u0(p, p.ns - 1) + p.nblk;
  p.cost = sy_tri(p.nblk);
  int64_t G = p.cost / (4 * (int64_t)ms);
  if (G > gmax) G = gmax;
  if (G < 1) G = 1;
  p.G = (int)G;
  p.Jt = 1;
  int Jt = 1;
  for (int g = 0; g < p.G; ++g) {
    const int64_t a = sy_start(p, g), b = sy_start(p, g + 1);
    if (a < b) {
      const int span = sy_strip(p, b - 1) - sy_strip(p, a) + 1;
      if (span > Jt) Jt = span;
    }
  }
  p.Jt = Jt;
  return p;
}

// the longest transposed list over the row tiles
inline int sy_max_tr_list(const SY& p) {
  int most = 0;
  for (int R = 1; R < p.nblk; ++R) {
    const int c = sy_tr_list(p, R, nullptr, 0);
    if (c > most) most = c;
  }
  return most;
}

}  // namespace ld
