// sync.hip -- ghost refill, 2:1 prolongation and restriction between the
// patches of a plan (rules in sync.hpp): the host builds the point maps once
// per plan, the kernel replays them after every Runge-Kutta stage.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>

#include "sync.hpp"

namespace chemora {

namespace {

// Lagrange weights of the midpoint between offsets 0 and 1 from the p
// points at offsets -p/2+1 .. p/2 (exact binary fractions)
template <int ORDER>
struct Mid;
template <>
struct Mid<4> {
  static __device__ __forceinline__ double w(int c) {
    const double t[4] = {-1.0 / 16, 9.0 / 16, 9.0 / 16, -1.0 / 16};
    return t[c];
  }
};
template <>
struct Mid<8> {
  static __device__ __forceinline__ double w(int c) {
    const double t[8] = {-5.0 / 2048, 49.0 / 2048, -245.0 / 2048, 1225.0 / 2048,
                         1225.0 / 2048, -245.0 / 2048, 49.0 / 2048, -5.0 / 2048};
    return t[c];
  }
};

// Copies (mid == 0): one work-item per item, all 24 grid functions -- the
// item is read once and its 24 loads are in flight together.  Consecutive
// work-items take consecutive items (destination memory order).
__global__ __launch_bounds__(256) void sync_copy_kernel(const SyncItem* __restrict__ items, int n,
                                                        double* const* __restrict__ bufs,
                                                        const SyncGeo* __restrict__ geo) {
  constexpr int NF = CHEMORA_NGF;
  const int t = blockIdx.x * 256 + threadIdx.x;
  if (t >= n) return;
  const SyncItem it = items[t];
  const int64_t sfs = geo[it.src].sf, sfd = geo[it.dst].sf;
  const double* src = bufs[it.src] + it.src_off;
  double* dst = bufs[it.dst] + it.dst_off;
  double v[NF];
#pragma unroll
  for (int f = 0; f < NF; ++f) v[f] = src[f * sfs];
#pragma unroll
  for (int f = 0; f < NF; ++f) dst[f * sfd] = v[f];
}

// Interpolations: one work-item per (item, grid function), blockIdx.y the
// grid function -- up to ORDER^3 taps each, so spread over 24 times as many
// work-items as items rather than summed in one.
template <int ORDER>
__global__ __launch_bounds__(256) void sync_interp_kernel(const SyncItem* __restrict__ items, int n,
                                                          double* const* __restrict__ bufs,
                                                          const SyncGeo* __restrict__ geo) {
  const int t = blockIdx.x * 256 + threadIdx.x;
  if (t >= n) return;
  const int f = blockIdx.y;
  const SyncItem it = items[t];
  const SyncGeo gs = geo[it.src], gd = geo[it.dst];
  const double* src = bufs[it.src] + f * gs.sf + it.src_off;
  const int n0 = (it.mid & 1) ? ORDER : 1, n1 = (it.mid & 2) ? ORDER : 1, n2 = (it.mid & 4) ? ORDER : 1;
  double acc = 0.0;
  for (int c2 = 0; c2 < n2; ++c2)
    for (int c1 = 0; c1 < n1; ++c1)
      for (int c0 = 0; c0 < n0; ++c0) {
        const double w = (n0 > 1 ? Mid<ORDER>::w(c0) : 1.0) * (n1 > 1 ? Mid<ORDER>::w(c1) : 1.0) *
                         (n2 > 1 ? Mid<ORDER>::w(c2) : 1.0);
        acc += w * src[c2 * gs.sz + c1 * gs.sy + c0];
      }
  bufs[it.dst][f * gd.sf + it.dst_off] = acc;
}

struct Box {
  int64_t lo[3], hi[3];   // inclusive global index ranges on one level
};

struct HostPatch {
  int level;
  int64_t I0[3];          // global index of interior point (0,0,0)
  Box interior, stored;
  int64_t sy, sz;
  int g;
};

bool contains(const Box& b, const int64_t* I) {
  for (int a = 0; a < 3; ++a)
    if (I[a] < b.lo[a] || I[a] > b.hi[a]) return false;
  return true;
}

bool overlaps(const Box& x, const Box& y) {
  for (int a = 0; a < 3; ++a)
    if (x.hi[a] < y.lo[a] || y.hi[a] < x.lo[a]) return false;
  return true;
}

int64_t offset(const HostPatch& P, const int64_t* I) {
  return (I[2] - P.I0[2] + P.g) * P.sz + (I[1] - P.I0[1] + P.g) * P.sy + (I[0] - P.I0[0] + P.g);
}

}  // namespace

int build_sync_maps(const chemora_params* P, const chemora_patch* X, int np, SyncMaps* out, std::string* err) {
  char buf[256];
  auto bad = [&](const char* m) {
    *err = m;
    return CHEMORA_EINVAL;
  };
  if (np < 1) return bad("no patches");
  double h0 = 0.0;
  for (int p = 0; p < np; ++p) h0 = std::max(h0, X[p].h);
  std::vector<HostPatch> H(np);
  int first = -1, maxL = 0;
  for (int p = 0; p < np; ++p) {
    const int L = (int)std::lround(std::log2(h0 / X[p].h));
    if (L < 0 || L > 20 || std::fabs(std::ldexp(h0, -L) - X[p].h) > 1e-12 * X[p].h) {
      std::snprintf(buf, sizeof buf, "patch %d: spacing %.17g is not the coarsest %.17g / 2^L", p, X[p].h, h0);
      return bad(buf);
    }
    H[p].level = L;
    maxL = std::max(maxL, L);
    if (L == 0 && first < 0) first = p;
  }
  for (int p = 0; p < np; ++p) {
    HostPatch& Q = H[p];
    Q.g = P->ghost;
    Q.sy = X[p].sy;
    Q.sz = X[p].sz;
    for (int a = 0; a < 3; ++a) {
      const double q = (X[p].origin[a] - X[first].origin[a]) / X[p].h;
      const int64_t I = (int64_t)std::llround(q);
      if (!std::isfinite(q) || std::fabs(q - (double)I) > 1e-9) {
        std::snprintf(buf, sizeof buf, "patch %d: origin off its level's lattice along axis %d", p, a);
        return bad(buf);
      }
      Q.I0[a] = I;
      Q.interior.lo[a] = I;
      Q.interior.hi[a] = I + X[p].n[a] - 1;
      Q.stored.lo[a] = I - Q.g;
      Q.stored.hi[a] = I + X[p].n[a] - 1 + Q.g;
    }
  }
  const int m = P->fd_order / 2;
  SyncMaps M;
  M.nlevels = maxL + 1;
  M.level.resize(np);
  for (int p = 0; p < np; ++p) M.level[p] = H[p].level;
  M.fill_start.push_back(0);
  for (int L = 0; L <= maxL; ++L) {
    for (int p = 0; p < np; ++p) {
      const HostPatch& Pp = H[p];
      if (Pp.level != L) continue;
      // candidate sources: same-level patches whose interior meets p's
      // stored box, coarse patches whose stored box meets it
      std::vector<int> same, coarse;
      for (int q = 0; q < np; ++q) {
        if (q == p) continue;
        if (H[q].level == L && overlaps(H[q].interior, Pp.stored)) same.push_back(q);
        if (H[q].level == L - 1) {
          Box c;
          for (int a = 0; a < 3; ++a) {
            c.lo[a] = 2 * H[q].stored.lo[a];
            c.hi[a] = 2 * H[q].stored.hi[a];
          }
          if (overlaps(c, Pp.stored)) coarse.push_back(q);
        }
      }
      const int g = Pp.g;
      for (int k = -g; k < X[p].n[2] + g; ++k)
        for (int j = -g; j < X[p].n[1] + g; ++j)
          for (int i = -g; i < X[p].n[0] + g; ++i) {
            if (i >= 0 && i < X[p].n[0] && j >= 0 && j < X[p].n[1] && k >= 0 && k < X[p].n[2]) continue;
            const int64_t gI[3] = {Pp.I0[0] + i, Pp.I0[1] + j, Pp.I0[2] + k};
            SyncItem it;
            it.dst = p;
            it.pad = 0;
            it.dst_off = offset(Pp, gI);
            int src = -1;
            for (int q : same)
              if (contains(H[q].interior, gI)) {
                src = q;
                break;
              }
            if (src >= 0) {
              it.src = src;
              it.mid = 0;
              it.src_off = offset(H[src], gI);
              M.fill.push_back(it);
              continue;
            }
            if (L == 0) continue;   // outer boundary
            int64_t lo[3];
            Box need;
            int mid = 0;
            for (int a = 0; a < 3; ++a) {
              const bool odd = ((gI[a] % 2) + 2) % 2 == 1;
              if (odd) {
                const int64_t left = (gI[a] - 1) / 2;
                lo[a] = left - m + 1;
                need.hi[a] = left + m;
                mid |= 1 << a;
              } else {
                lo[a] = gI[a] / 2;
                need.hi[a] = lo[a];
              }
              need.lo[a] = lo[a];
            }
            for (int q : coarse)
              if (contains(H[q].stored, need.lo) && contains(H[q].stored, need.hi)) {
                src = q;
                break;
              }
            if (src < 0) {
              std::snprintf(buf, sizeof buf,
                            "patch %d (level %d): ghost point (%d, %d, %d) is in no patch of its level and no "
                            "patch of the next coarser level holds its interpolation stencil",
                            p, L, i, j, k);
              return bad(buf);
            }
            it.src = src;
            it.mid = mid;
            it.src_off = offset(H[src], lo);
            M.fill.push_back(it);
          }
    }
    // within the level, the items grouped by their stencil (copies first,
    // then by the set of midpoint axes) and kept in destination order inside
    // a group: a wave then runs one loop shape, without divergence
    std::stable_sort(M.fill.begin() + M.fill_start.back(), M.fill.end(),
                     [](const SyncItem& x, const SyncItem& y) { return x.mid < y.mid; });
    M.fill_copies.push_back((int)(std::find_if(M.fill.begin() + M.fill_start.back(), M.fill.end(),
                                               [](const SyncItem& x) { return x.mid != 0; }) -
                                  (M.fill.begin() + M.fill_start.back())));
    M.fill_start.push_back((int)M.fill.size());
  }
  // restriction, finest pair first
  M.restr_start.push_back(0);
  for (int L = maxL; L >= 1; --L) {
    for (int c = 0; c < np; ++c) {
      const HostPatch& C = H[c];
      if (C.level != L - 1) continue;
      std::vector<int> fine;
      for (int q = 0; q < np; ++q) {
        if (H[q].level != L) continue;
        Box b;
        for (int a = 0; a < 3; ++a) {
          b.lo[a] = 2 * C.interior.lo[a];
          b.hi[a] = 2 * C.interior.hi[a];
        }
        if (overlaps(b, H[q].interior)) fine.push_back(q);
      }
      if (fine.empty()) continue;
      for (int k = 0; k < X[c].n[2]; ++k)
        for (int j = 0; j < X[c].n[1]; ++j)
          for (int i = 0; i < X[c].n[0]; ++i) {
            const int64_t cI[3] = {C.I0[0] + i, C.I0[1] + j, C.I0[2] + k};
            const int64_t fI[3] = {2 * cI[0], 2 * cI[1], 2 * cI[2]};
            for (int q : fine)
              if (contains(H[q].interior, fI)) {
                SyncItem it;
                it.dst = c;
                it.src = q;
                it.mid = 0;
                it.pad = 0;
                it.dst_off = offset(C, cI);
                it.src_off = offset(H[q], fI);
                M.restr.push_back(it);
                break;
              }
          }
    }
    M.restr_start.push_back((int)M.restr.size());
  }
  if (M.fill.size() > (size_t)INT32_MAX || M.restr.size() > (size_t)INT32_MAX) return bad("too many ghost points");
  *out = std::move(M);
  return CHEMORA_OK;
}

void launch_sync(int order, const SyncItem* items, int n, int ncopy, double* const* bufs, const SyncGeo* geo,
                 hipStream_t s) {
  if (ncopy > 0)
    hipLaunchKernelGGL(sync_copy_kernel, dim3((ncopy + 255) / 256), dim3(256), 0, s, items, ncopy, bufs, geo);
  const int ni = n - ncopy;
  if (ni <= 0) return;
  dim3 grid((ni + 255) / 256, CHEMORA_NGF, 1);
  if (order == 8)
    hipLaunchKernelGGL(sync_interp_kernel<8>, grid, dim3(256), 0, s, items + ncopy, ni, bufs, geo);
  else
    hipLaunchKernelGGL(sync_interp_kernel<4>, grid, dim3(256), 0, s, items + ncopy, ni, bufs, geo);
}

}  // namespace chemora
