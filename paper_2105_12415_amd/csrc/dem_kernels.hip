// HIP kernels (gfx950) and the C ABI of the contact-detection path.
//
// Step of one dem_find_contacts call (all on the caller's stream):
//   k_reset    clear the device counters (a kernel, not a memset, so the
//              call can be captured in a graph and replayed)
//   k_flatten  world vertices -> triangle soup (Section 3, triangle soup
//              implementation note: per-triangle coordinates with no
//              indirection), plus the regularised Newton diagonal
//   k_seed     one work item per (root-range x root-range) chunk of each
//              candidate particle pair (HIER) or per fine tile (FLAT)
//   k_level    HIER: one launch per tree depth; every item is a product of
//              two child ranges; each child pair runs the fixed-count
//              iteration + lower bound; surviving surrogate pairs become the
//              next depth's items, fine pairs that are not pruned go to the
//              near list (Algorithm 5, pairwise form)
//   k_flat     FLAT: LDS-staged tiles over all fine pairs (Algorithm 2)
//   k_near     exact comparison-based distance for the near list, contact
//              emission and the penalty energy (Algorithm 4, fallback part)
// dem_contact_backward launches k_backward: recompute closest points per
// contact and scatter the energy gradient with atomics.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <type_traits>

#include "dem.h"
#include "dem_geom.hpp"

using namespace dem;

namespace {

constexpr int kWave = 64;

// ------------------------------------------------------------------ layout
// Soup record: 12 values + 4 ints.  float: 64 B (one half cache line),
// double: 112 B.
template <typename T>
struct alignas(16) SoupRec {
  T g[12];         // v0.xyz eps | e1.xyz ia | e2.xyz ib
  int32_t topo[4]; // child_begin, child_count, size bound (float bits), particle (last: the
                   // descent does not read it, so the three words it reads are contiguous)
};

// Bit of topo[1] (above the child count) marking a surrogate whose children
// are fine triangles.
constexpr int kKidsFine = 1 << 16;
constexpr int kCountMask = 0xFFFF;

// Every work list is split into kSeg segments with a tail counter each; a
// block appends to segment blockIdx % kSeg (its XCD under round-robin
// dispatch).  Appends from all compute units to one tail serialise in the
// memory-side atomic unit; eight tails spread them.
constexpr int kSeg = 8;
// XCC (XCD) ids the hardware can report: the low 4 bits of HW_REG_XCC_ID.
constexpr int kMaxXcc = 16;
constexpr int kFinePart = 64;

// Statistics and energy of the forward pass in kStatPart partial sums: a
// block adds its block-reduced counts to partial blockIdx % kStatPart, each
// partial on lines of its own, and k_fold_stats sums the partials into
// dem_stats and the energy after the call's last kernel.  (One atomic per
// wave on one address serialises in L2 at the end of every launch: about
// 10 % of the descent.)
constexpr int kStatPart = 16;
struct alignas(128) StatPart {
  unsigned long long evals[DEM_MAX_LEVELS];
  unsigned long long survivors[DEM_MAX_LEVELS];
  unsigned long long near, fallback, contacts, certified;
  double energy;
};

struct Counters {
  uint32_t tail[DEM_MAX_LEVELS + 1][kSeg];  // level queues
  uint32_t near_tail[kSeg];                 // fine pairs not pruned
  uint32_t fb_tail[kSeg];                   // pairs the certificate could not settle
  uint32_t fr_unfold;                       // frontier step: leaves that widen
  uint32_t fr_collapse;                     // frontier step: sibling groups that narrow
  uint32_t fr_skip;                         // frontier step: leave the active sets as they are
  uint32_t claim[DEM_MAX_LEVELS][kSeg];     // persistent descent: batches claimed per depth and segment
  // persistent descent: grid barrier, every counter on a 128-byte line of its
  // own (arrivals at one address serialise; these spread them)
  alignas(128) uint32_t bar_top[32];        // arrivals of whole XCCs, summed over the call's barriers
  uint32_t bar_reg_top[32];                 // registration groups complete
  uint32_t bar_reg[kSeg][32];               // registrations per group of blocks (blockIdx % kSeg)
  uint32_t bar_blocks[kMaxXcc][32];         // blocks resident on each XCC
  uint32_t bar_arrive[kMaxXcc][32];         // block arrivals per XCC, summed over the call's barriers
  uint32_t bar_release[kMaxXcc][32];        // barriers the XCC's last block has released
  // statistics: records written by the lazy flattening, in kFinePart partial
  // counts on lines of their own (folded into dem_stats by the exact pass)
  uint32_t fine_part[kFinePart][32];
  StatPart stat_part[kStatPart];
};

constexpr size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

struct WsLayout {
  size_t ctr, soup, mark, qa, qb, near_, fb, total;
};

WsLayout ws_layout(int precision, int64_t n_tris, int64_t qcap, int64_t ncap) {
  WsLayout L;
  size_t rec = precision == DEM_F64 ? sizeof(SoupRec<double>) : sizeof(SoupRec<float>);
  size_t o = 0;
  L.ctr = o; o = align_up(o + sizeof(Counters), 256);
  L.soup = o; o = align_up(o + rec * (size_t)n_tris, 256);
  L.mark = o; o = align_up(o + (size_t)n_tris, 256);
  L.qa = o; o = align_up(o + 16 * (size_t)qcap, 256);
  L.qb = o; o = align_up(o + 16 * (size_t)qcap, 256);
  L.near_ = o; o = align_up(o + 8 * (size_t)ncap, 256);
  L.fb = o; o = align_up(o + 8 * (size_t)ncap, 256);
  L.total = o;
  return L;
}

// Soup record t: the triangle, its child range, particle and whether its
// children are fine.
template <typename T>
__device__ __forceinline__ Tri<T> load_tri(const SoupRec<T>* __restrict__ s, int t, int& cb, int& cc,
                                           int& part, bool& kids_fine) {
  // 32-bit byte offset from a uniform base (soups stay below 4 GiB)
  const char* rp = reinterpret_cast<const char*>(s) + (uint32_t)t * (uint32_t)sizeof(SoupRec<T>);
  Tri<T> x;
  int4 d;
  if constexpr (sizeof(T) == 4) {
    const float4* p = reinterpret_cast<const float4*>(rp);
    float4 a = p[0], b = p[1], c = p[2];
    d = reinterpret_cast<const int4*>(rp)[3];
    x.v0 = {a.x, a.y, a.z}; x.eps = a.w;
    x.e1 = {b.x, b.y, b.z}; x.ia = b.w;
    x.e2 = {c.x, c.y, c.z}; x.ib = c.w;
  } else {
    const double2* p = reinterpret_cast<const double2*>(rp);
    double2 a0 = p[0], a1 = p[1], b0 = p[2], b1 = p[3], c0 = p[4], c1 = p[5];
    d = reinterpret_cast<const int4*>(rp)[6];
    x.v0 = {a0.x, a0.y, a1.x}; x.eps = a1.y;
    x.e1 = {b0.x, b0.y, b1.x}; x.ia = b1.y;
    x.e2 = {c0.x, c0.y, c1.x}; x.ib = c1.y;
  }
  cb = d.x; cc = d.y & kCountMask; part = d.w;
  kids_fine = (d.y & kKidsFine) != 0;
  x.size = T(__int_as_float(d.z));
  return x;
}

template <typename T>
__device__ __forceinline__ Tri<T> load_tri(const SoupRec<T>* __restrict__ s, int t, int& cb, int& cc,
                                           int& part) {
  bool kf;
  return load_tri(s, t, cb, cc, part, kf);
}

__device__ __forceinline__ int lane_id() { return __lane_id(); }

// Wave-aggregated append: one atomic per wave; returns this lane's slot.
// Must be called by every lane that may append (pred false for the rest).
__device__ __forceinline__ uint32_t wave_append(bool pred, uint32_t* tail, uint32_t& slot_ok) {
  unsigned long long m = __ballot(pred);
  slot_ok = 0;
  if (m == 0ull) return 0;
  int leader = __ffsll((long long)m) - 1;
  uint32_t base = 0;
  if (lane_id() == leader) base = atomicAdd(tail, (uint32_t)__popcll(m));
  base = __shfl(base, leader);
  unsigned long long lt = (lane_id() == 0) ? 0ull : (~0ull >> (64 - lane_id()));
  slot_ok = pred ? 1u : 0u;
  return base + (uint32_t)__popcll(m & lt);
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// Block sums of NV counts (every thread calls; valid in thread 0).
template <int NV>
__device__ __forceinline__ void block_sums(unsigned long long (&v)[NV]) {
  __shared__ unsigned long long red[NV][16];
  const int w = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    v[k] = wave_sum_u64(v[k]);
    if (lane_id() == 0) red[k][w] = v[k];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      unsigned long long t = 0;
      for (int q = 0; q < nw; ++q) t += red[k][q];
      v[k] = t;
    }
  }
  __syncthreads();
}

__device__ __forceinline__ double block_sum_f64(double v) {
  __shared__ double redd[16];
  const int w = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
  v = wave_sum(v);
  if (lane_id() == 0) redd[w] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int q = 0; q < nw; ++q) t += redd[q];
    v = t;
  }
  __syncthreads();
  return v;
}

template <typename V>
__device__ __forceinline__ V wave_min(V v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o));
  return v;
}

template <typename V>
__device__ __forceinline__ V wave_max(V v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o));
  return v;
}

__device__ __forceinline__ void add_stat(unsigned long long* p, unsigned long long v) {
  if (p) atomicAdd(p, v);
}

// ------------------------------------------------------------------ kernels
__global__ void k_reset(Counters* ctr, dem_stats* stats, uint32_t* status, uint32_t* count,
                        double* energy) {
  int t = threadIdx.x;
  uint32_t* c = reinterpret_cast<uint32_t*>(ctr);
  for (int i = t; i < (int)(sizeof(Counters) / 4); i += blockDim.x) c[i] = 0;
  if (stats) {
    unsigned long long* s = reinterpret_cast<unsigned long long*>(stats);
    for (int i = t; i < (int)(sizeof(dem_stats) / 8); i += blockDim.x) s[i] = 0;
  }
  if (t == 0) {
    *status = 0;
    *count = 0;
    if (energy) *energy = 0.0;
  }
}

// Sums of the forward's partial statistics and energy (one wave, after the
// call's last kernel).
__global__ void k_fold_stats(const StatPart* part, const uint32_t* fine_part, int n_levels, dem_stats* stats,
                             double* energy) {
  const int t = threadIdx.x;
  if (stats) {
    for (int d = t; d < n_levels && d < DEM_MAX_LEVELS; d += blockDim.x) {
      unsigned long long e = 0, v = 0;
      for (int q = 0; q < kStatPart; ++q) {
        e += part[q].evals[d];
        v += part[q].survivors[d];
      }
      if (e) stats->evals[d] += e;
      if (v) stats->survivors[d] += v;
    }
    if (t == 0) {
      unsigned long long nr = 0, fb = 0, ct = 0, ce = 0;
      for (int q = 0; q < kStatPart; ++q) {
        nr += part[q].near;
        fb += part[q].fallback;
        ct += part[q].contacts;
        ce += part[q].certified;
      }
      stats->near += nr;
      stats->fallback += fb;
      stats->contacts += ct;
      stats->certified += ce;
      unsigned long long fr = 0;
      for (int q = 0; q < kFinePart; ++q) fr += fine_part[q * 32];
      stats->fine_records += fr;
    }
  }
  if (energy && t == 1) {
    double e = 0.0;
    for (int q = 0; q < kStatPart; ++q) e += part[q].energy;
    *energy += e;
  }
}

__global__ void k_zero_scalar(double* e) {
  if (threadIdx.x == 0) *e = 0.0;
}

// Flattening inputs (the scene's static arrays, the step's pose, the soup).
template <typename T>
struct FlatArgs {
  const T* verts;
  int n_verts;
  const int32_t* tv;
  int n_tris;
  const int32_t* cbeg;
  const int32_t* ccnt;
  const int32_t* tpart;
  const T* teps;
  const T* pose;
  T areg_rel;
  T omega;
  const int32_t* root_begin;
  const int32_t* root_count;
  const int32_t* fine_begin;
  SoupRec<T>* soup;
  uint8_t* mark;  // lazy mode: per-surrogate "a pair with it survived" flags
  int lazy;
  uint32_t* status;
  uint32_t* fine_part;  // statistics: Counters::fine_part (or null)
};

// Soup record of triangle t: world vertices (pose applied), edges, the
// regularised Newton diagonal and the topology word.
template <typename T>
__device__ __forceinline__ SoupRec<T> flatten_rec(const FlatArgs<T>& a, int t, int cb, int cc, int part) {
  const T* X = a.verts;
  const T* Y = a.verts + a.n_verts;
  const T* Z = a.verts + 2 * (size_t)a.n_verts;
  int i0 = a.tv[t], i1 = a.tv[a.n_tris + t], i2 = a.tv[2 * (size_t)a.n_tris + t];
  V3<T> v0 = {X[i0], Y[i0], Z[i0]};
  V3<T> v1 = {X[i1], Y[i1], Z[i1]};
  V3<T> v2 = {X[i2], Y[i2], Z[i2]};
  V3<T> e1 = v1 - v0, e2 = v2 - v0;
  if (a.pose) {
    // rigid motion of the particle applied while flattening: world = R v + c
    const T* P = a.pose + 12 * (size_t)part;
    V3<T> r0 = {P[0], P[1], P[2]}, r1 = {P[3], P[4], P[5]}, r2 = {P[6], P[7], P[8]};
    V3<T> c = {P[9], P[10], P[11]};
    v0 = V3<T>{dot(r0, v0), dot(r1, v0), dot(r2, v0)} + c;
    e1 = V3<T>{dot(r0, e1), dot(r1, e1), dot(r2, e1)};
    e2 = V3<T>{dot(r0, e2), dot(r1, e2), dot(r2, e2)};
  }
  T ia, ib;
  newton_steps(e1, e2, a.areg_rel, a.omega, ia, ib);
  SoupRec<T> r;
  r.g[0] = v0.x; r.g[1] = v0.y; r.g[2] = v0.z; r.g[3] = a.teps[t];
  r.g[4] = e1.x; r.g[5] = e1.y; r.g[6] = e1.z; r.g[7] = ia;
  r.g[8] = e2.x; r.g[9] = e2.y; r.g[10] = e2.z; r.g[11] = ib;
  // size bound, rounded up when narrowed to float
  const float sz = (float)(tri_size(e1, e2) * T(1.0 + 1.0 / 1048576.0));
  // children of the last surrogate level start at the particle's fine range
  const bool kids_fine = cc > 0 && cb >= a.fine_begin[part];
  r.topo[0] = cb; r.topo[1] = cc | (kids_fine ? kKidsFine : 0); r.topo[2] = __float_as_int(sz);
  r.topo[3] = part;
  T chk = v0.x + v0.y + v0.z + e1.x + e1.y + e1.z + e2.x + e2.y + e2.z;
  if (!isfinite(chk)) atomicOr(a.status, DEM_DEV_NONFINITE);
  return r;
}

template <typename T>
__device__ __forceinline__ void flatten_one(const FlatArgs<T>& a, int t, int cb, int cc, int part) {
  a.soup[t] = flatten_rec(a, t, cb, cc, part);
}

// Every triangle (eager), or the surrogates and root triangles only (lazy:
// fine children are written by k_fine once a pair with their parent
// survives).  Lazy mode also clears the surrogates' survival flags.
// The block's records go through LDS so that the stores leave as whole
// contiguous 16-byte chunks of the block's output range (a record per lane
// would scatter each store instruction over 64 lines).  Launched with
// kFlatBlock threads per block.
constexpr int kFlatBlock = 256;

template <typename T>
__global__ void __launch_bounds__(kFlatBlock) k_flatten(FlatArgs<T> a) {
  __shared__ SoupRec<T> stage[kFlatBlock];
  __shared__ uint8_t act[kFlatBlock];
  const int t = blockIdx.x * kFlatBlock + threadIdx.x;
  // every input vertex is checked once per step, also the vertices of fine
  // triangles below pruned surrogates that no record reads this step
  for (int v = t; v < a.n_verts; v += gridDim.x * kFlatBlock) {
    const T vx = a.verts[v], vy = a.verts[a.n_verts + v], vz = a.verts[2 * (size_t)a.n_verts + v];
    if (!(isfinite(vx) && isfinite(vy) && isfinite(vz))) atomicOr(a.status, DEM_DEV_NONFINITE);
  }
  bool on = t < a.n_tris;
  if (on) {
    const int cc = a.ccnt[t];
    if (cc < 0 || cc > DEM_MAX_CHILDREN) atomicOr(a.status, DEM_DEV_BAD_TREE);
    const int part = a.tpart[t];
    if (a.lazy) {
      if (cc > 0) a.mark[t] = 0;
      else if ((uint32_t)(t - a.root_begin[part]) >= (uint32_t)a.root_count[part]) on = false;  // fine, below a surrogate
    }
    if (on) stage[threadIdx.x] = flatten_rec(a, t, a.cbeg[t], cc, part);
  }
  act[threadIdx.x] = on ? 1 : 0;
  __syncthreads();
  constexpr int kChunks = (int)(sizeof(SoupRec<T>) / 16);
  static_assert(sizeof(SoupRec<T>) % 16 == 0, "16-byte chunks");
  const uint4* src = reinterpret_cast<const uint4*>(stage);
  uint4* dst = reinterpret_cast<uint4*>(a.soup + (size_t)blockIdx.x * kFlatBlock);
  for (int c = threadIdx.x; c < kFlatBlock * kChunks; c += kFlatBlock)
    if (act[c / kChunks]) dst[c] = src[c];
}

// Block-wide exclusive scan of v (blockDim <= 1024) into offs[0..n].
__device__ __forceinline__ void block_scan(int v, int* offs, int* wsum, int n) {
  int lane = lane_id();
  int wid = threadIdx.x / kWave;
  int x = v;
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    int y = __shfl_up(x, o);
    if (lane >= o) x += y;
  }
  if (lane == kWave - 1) wsum[wid] = x;
  __syncthreads();
  if (threadIdx.x == 0) {
    int acc = 0;
    int nw = (blockDim.x + kWave - 1) / kWave;
    for (int w = 0; w < nw; ++w) {
      int s = wsum[w];
      wsum[w] = acc;
      acc += s;
    }
    offs[n] = acc;  // total lives after the last item (read only after sync)
  }
  __syncthreads();
  if ((int)threadIdx.x < n) offs[threadIdx.x] = x - v + wsum[wid];
  __syncthreads();
}

// Lazy mode, after the descent at depth d: the children of every depth-d
// surrogate (parents[0 .. n)) that survived in some pair are written.  A
// thread tests one parent's mark; a block-wide scan then packs the children
// of the marked parents onto consecutive lanes (most parents are not
// marked: testing four lanes per parent left most lanes of the flattening
// idle), and the block's records go through LDS so that sibling records
// leave as whole 16-byte chunks, as in k_flatten.
template <typename T>
struct FineShared {
  SoupRec<T> stage[kFlatBlock];
  int dest[kFlatBlock];
  int offs[kFlatBlock + 1];                      // child slots of the block's parents
  int wsum[16];
  int cb[kFlatBlock];                            // child range begin of each parent
  uint8_t owner[kFlatBlock * DEM_MAX_CHILDREN];  // child slot -> parent (thread)
};

// The children of parents[0 .. n) that survived (mark set), over blocks
// start, start + stride, ... of kFlatBlock parents.
template <typename T>
__device__ __forceinline__ void fine_range(const FlatArgs<T>& a, const int32_t* __restrict__ parents, int n,
                                           FineShared<T>& sh, uint32_t start, uint32_t stride) {
  uint32_t written = 0;  // records of the parents this thread found marked
  for (int64_t base = start * (int64_t)kFlatBlock; base < n; base += (int64_t)stride * kFlatBlock) {
    const int64_t i = base + threadIdx.x;
    int cb = 0, cc = 0;
    if (i < n) {
      const int s = parents[i];
      if ((uint32_t)s >= (uint32_t)a.n_tris) {
        atomicOr(a.status, DEM_DEV_BAD_TREE);
      } else if (a.mark[s]) {
        cb = a.cbeg[s];
        cc = a.ccnt[s];
        if (cc < 1 || cc > DEM_MAX_CHILDREN || cb < 0 || cb > a.n_tris - cc) {
          atomicOr(a.status, DEM_DEV_BAD_TREE);
          cc = 0;
        }
      }
    }
    written += (uint32_t)cc;
    block_scan(cc, sh.offs, sh.wsum, kFlatBlock);
    sh.cb[threadIdx.x] = cb;
    for (int q = 0; q < cc; ++q) sh.owner[sh.offs[threadIdx.x] + q] = (uint8_t)threadIdx.x;
    __syncthreads();
    const int total = sh.offs[kFlatBlock];
    for (int k0 = 0; k0 < total; k0 += kFlatBlock) {
      const int k = k0 + (int)threadIdx.x;
      int d = -1;
      if (k < total) {
        const int pa = sh.owner[k];
        d = sh.cb[pa] + (k - sh.offs[pa]);
        sh.stage[threadIdx.x] = flatten_rec(a, d, a.cbeg[d], a.ccnt[d], a.tpart[d]);
      }
      sh.dest[threadIdx.x] = d;
      __syncthreads();
      constexpr int kChunks = (int)(sizeof(SoupRec<T>) / 16);
      const uint4* src = reinterpret_cast<const uint4*>(sh.stage);
      uint4* out = reinterpret_cast<uint4*>(a.soup);
      for (int c = threadIdx.x; c < kFlatBlock * kChunks; c += kFlatBlock) {
        const int dr = sh.dest[c / kChunks];
        if (dr >= 0) out[(size_t)dr * kChunks + c % kChunks] = src[c];
      }
      __syncthreads();
    }
  }
  if (a.fine_part) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) written += __shfl_xor(written, o);
    if (lane_id() == 0 && written)
      atomicAdd(&a.fine_part[((blockIdx.x * (kFlatBlock / 64) + threadIdx.x / 64) % kFinePart) * 32], written);
  }
}

template <typename T>
__global__ void __launch_bounds__(kFlatBlock) k_fine(FlatArgs<T> a, const int32_t* __restrict__ parents, int n) {
  __shared__ FineShared<T> sh;
  fine_range(a, parents, n, sh, blockIdx.x, gridDim.x);
}

// Items covering range_i x range_j of candidate pair pr in chunks, appended
// to segment blockIdx % kSeg of the level-0 list (block-level; base: a word
// of LDS).
__device__ __forceinline__ void seed_pair(int pr, const int32_t* __restrict__ pairs, int n_pairs,
                                          const int32_t* __restrict__ rbeg, const int32_t* __restrict__ rcnt,
                                          int ci, int cj, int4* __restrict__ q, uint32_t* tails, int64_t seg_cap,
                                          uint32_t* status, uint32_t& base) {
  int pi = pairs[pr], pj = pairs[n_pairs + pr];
  int bi = rbeg[pi], ni = rcnt[pi], bj = rbeg[pj], nj = rcnt[pj];
  int nci = (ni + ci - 1) / ci, ncj = (nj + cj - 1) / cj;
  int n = nci * ncj;
  const uint32_t x = blockIdx.x % kSeg;
  __syncthreads();
  if (threadIdx.x == 0) base = n > 0 ? atomicAdd(&tails[x], (uint32_t)n) : 0;
  __syncthreads();
  int4* seg = q + (size_t)x * (size_t)seg_cap;
  for (int k = threadIdx.x; k < n; k += blockDim.x) {
    int ii = k / ncj, jj = k - ii * ncj;
    int4 it;
    it.x = bi + ii * ci;
    it.y = min(ci, ni - ii * ci);
    it.z = bj + jj * cj;
    it.w = min(cj, nj - jj * cj);
    uint64_t slot = (uint64_t)base + (uint64_t)k;
    if (slot < (uint64_t)seg_cap)
      seg[slot] = it;
    else
      atomicOr(status, DEM_DEV_QUEUE_OVERFLOW);
  }
}

// One block per candidate pair.
__global__ void k_seed(const int32_t* __restrict__ pairs, int n_pairs,
                       const int32_t* __restrict__ rbeg, const int32_t* __restrict__ rcnt, int ci,
                       int cj, int4* __restrict__ q, uint32_t* tails, int64_t seg_cap,
                       uint32_t* status) {
  __shared__ uint32_t base;
  if ((int)blockIdx.x < n_pairs)
    seed_pair(blockIdx.x, pairs, n_pairs, rbeg, rcnt, ci, cj, q, tails, seg_cap, status, base);
}

struct LevelArgs {
  const int4* qin;
  const uint32_t* tail_in;   // [kSeg]
  int4* qout;
  uint32_t* tail_out;        // [kSeg]
  int64_t qcap;              // entries per segment
  int2* near_;
  uint32_t* near_tail;       // [kSeg]
  int64_t ncap;              // entries per segment
  dem_stats* stats;
  StatPart* part;            // partial statistics (with stats; null: straight into stats)
  uint32_t* status;
  int depth;
  int dense;
  int batch;
  uint8_t* mark;             // lazy flattening: survival flags of surrogates (else null)
  int half;                  // this depth runs the Newton iteration in half precision
  int deepest;               // the tree's deepest depth: a surrogate survivor there means a malformed tree
  IterParams ip;
};

// Block-local append buffer in LDS: lanes reserve slots with one LDS atomic
// per wave; the block flushes the buffer to the global queue with a single
// global atomic (same-address global atomics serialise in L2, so one per
// wave per evaluation round would dominate the descent).
template <typename R, int CAP>
struct LdsQueue {
  R buf[CAP];
  uint32_t n;
  uint32_t gbase;
};

// Slot of this lane in a wave-aggregated LDS append (valid where pred holds);
// false when no lane of the wave appends.
__device__ __forceinline__ bool lds_reserve(bool pred, uint32_t* n, uint32_t& slot) {
  unsigned long long m = __ballot(pred);
  if (m == 0ull) return false;
  int leader = __ffsll((long long)m) - 1;
  uint32_t base = 0;
  if (lane_id() == leader) base = atomicAdd(n, (uint32_t)__popcll(m));
  // the leader's slot to every lane with a lane read (no LDS permute)
  base = (uint32_t)__builtin_amdgcn_readlane((int)base, leader);
  unsigned long long lt = (lane_id() == 0) ? 0ull : (~0ull >> (64 - lane_id()));
  slot = base + (uint32_t)__popcll(m & lt);
  return true;
}

template <typename R>
__device__ __forceinline__ void lds_append(bool pred, R rec, R* buf, uint32_t* n) {
  uint32_t slot;
  if (lds_reserve(pred, n, slot) && pred) buf[slot] = rec;
}

__device__ __forceinline__ bool item_counts_ok(const int4& it) {
  return (uint32_t)(it.y - 1) < (uint32_t)DEM_MAX_CHILDREN && (uint32_t)(it.w - 1) < (uint32_t)DEM_MAX_CHILDREN;
}

// Survivor stage of the depths above the deepest.  In a round a lane
// appends at most one entry, a surrogate item or a near pair, never both, so
// the two lists share one pool: items from its front (first children as
// int2, both child counts - 1 in one byte), near pairs from its back.
template <int CAP>
struct SharedStage {
  int2 pool[CAP];
  uint8_t cnt[CAP];
  uint32_t ni, nn;  // items, near pairs
  uint32_t gi, gn;  // global bases of a flush
};

template <int CAP>
__device__ __forceinline__ void stage_reset(SharedStage<CAP>& q) { q.ni = 0; q.nn = 0; }
template <typename R, int CAP>
__device__ __forceinline__ void stage_reset(LdsQueue<R, CAP>& q) { q.n = 0; }

// Copy an LDS queue to global memory (whole block): one atomic on the tail of
// this block's segment reserves the range.  seg_cap = entries per segment.
template <typename R, int CAP>
__device__ __forceinline__ void lds_flush(LdsQueue<R, CAP>& q, uint32_t* tails, R* out, int64_t seg_cap,
                                          uint32_t* status, uint32_t flag) {
  const uint32_t x = blockIdx.x % kSeg;
  if (threadIdx.x == 0) q.gbase = q.n ? atomicAdd(&tails[x], q.n) : 0u;
  __syncthreads();
  const uint32_t n = q.n, g = q.gbase;
  R* seg = out + (size_t)x * (size_t)seg_cap;
  for (uint32_t k = threadIdx.x; k < n; k += blockDim.x) {
    uint64_t slot = (uint64_t)g + k;
    if (slot < (uint64_t)seg_cap) seg[slot] = q.buf[k];
    else atomicOr(status, flag);
  }
  __syncthreads();
  if (threadIdx.x == 0) q.n = 0;
  __syncthreads();
}

// Both lists of a shared stage to their segments of the next queue and of
// the near list (one atomic on each tail), then empty.
template <int CAP>
__device__ __forceinline__ void shared_flush(SharedStage<CAP>& q, uint32_t* qtails, int4* qout, int64_t qcap,
                                             uint32_t* ntails, int2* nout, int64_t ncap, uint32_t* status) {
  const uint32_t x = blockIdx.x % kSeg;
  if (threadIdx.x == 0) {
    q.gi = q.ni ? atomicAdd(&qtails[x], q.ni) : 0u;
    q.gn = q.nn ? atomicAdd(&ntails[x], q.nn) : 0u;
  }
  __syncthreads();
  const uint32_t ni = q.ni, nn = q.nn, gi = q.gi, gn = q.gn;
  int4* qseg = qout + (size_t)x * (size_t)qcap;
  int2* nseg = nout + (size_t)x * (size_t)ncap;
  for (uint32_t k = threadIdx.x; k < ni; k += blockDim.x) {
    const uint64_t slot = (uint64_t)gi + k;
    const int2 f = q.pool[k];
    const int c = q.cnt[k];
    if (slot < (uint64_t)qcap) qseg[slot] = make_int4(f.x, (c >> 4) + 1, f.y, (c & 15) + 1);
    else atomicOr(status, DEM_DEV_QUEUE_OVERFLOW);
  }
  for (uint32_t k = threadIdx.x; k < nn; k += blockDim.x) {
    const uint64_t slot = (uint64_t)gn + k;
    if (slot < (uint64_t)ncap) nseg[slot] = q.pool[CAP - 1 - k];
    else atomicOr(status, DEM_DEV_NEAR_OVERFLOW);
  }
  __syncthreads();
  if (threadIdx.x == 0) { q.ni = 0; q.nn = 0; }
  __syncthreads();
}

// Consumer side of a segmented list: prefix of the segment fills.
struct SegView {
  uint32_t pre[kSeg + 1];
};

__device__ __forceinline__ void seg_view(SegView& v, const uint32_t* tails, int64_t seg_cap) {
  if (threadIdx.x == 0) {
    uint32_t acc = 0;
    v.pre[0] = 0;
    for (int x = 0; x < kSeg; ++x) {
      acc += (uint32_t)min((uint64_t)tails[x], (uint64_t)seg_cap);
      v.pre[x + 1] = acc;
    }
  }
  __syncthreads();
}

// Storage index of the i-th entry (i < v.pre[kSeg]).
__device__ __forceinline__ size_t seg_index(const SegView& v, uint32_t i, int64_t seg_cap) {
  int x = 0;
#pragma unroll
  for (int k = 1; k < kSeg; ++k) x += (i >= v.pre[k]) ? 1 : 0;
  return (size_t)x * (size_t)seg_cap + (i - v.pre[x]);
}

constexpr int kStageNear = 512;
constexpr int kStageFlat = 2048;  // >= 4 evaluation rounds of 256 lanes between checks

// Outcome of a frontier leaf in a step (byte 0 of its outcome word).
constexpr uint32_t kOutPrune = 0, kOutKeep = 1, kOutUnfold = 2, kOutNear = 3;

// LDS of the descent over one depth: one item per thread, and a survivor
// stage for kRounds evaluation rounds between stage checks (each check is a
// block barrier; fewer checks measured faster than more waves per SIMD).
// At BLOCK = 256: 28.7 KB above the deepest depth (the shared stage, five
// blocks per CU), 26.4 KB at the deepest (near pairs only, six blocks).
#ifndef DEM_LEVEL_ROUNDS
#define DEM_LEVEL_ROUNDS 8
#endif
#ifndef DEM_LEAF_ROUNDS
#define DEM_LEAF_ROUNDS 8
#endif
template <int BLOCK, bool LEAF = false>
struct LevelShared {
  static constexpr int kRounds = LEAF ? DEM_LEAF_ROUNDS : DEM_LEVEL_ROUNDS;  // evaluation rounds between stage checks
  static constexpr int kCap = (kRounds + 1) * BLOCK;
  int4 items[BLOCK];
  int offs[BLOCK + 1];
  int wsum[16];
  uint8_t owner[BLOCK * 8];
  // the deepest depth stages near pairs only
  std::conditional_t<LEAF, LdsQueue<int2, kCap>, SharedStage<kCap>> st;
  SegView view;
  uint32_t claim;      // persistent descent: the next batch claimed by thread 0
  uint32_t claim_seg;  // persistent descent: the segment of that batch
};

struct LevelCounts {
  uint32_t evals, surv, near;  // per lane and depth (summed in 64 bits at the depth's end)
};

// One batch of work items: items [first, first + n) of segment x of the
// depth's queue.  Work items are products of two triangle ranges (the
// children of a surviving surrogate pair, or a chunk of the roots); lanes
// take one child pair each, located through a block-wide scan of the items'
// pair counts.  Survivors are staged in LDS and flushed to the block's own
// segment of the next queue / the near list.
//
// LEAF: the deepest tree depth, where every record is a fine triangle (a
// surrogate that reaches depth d sits on tree level d, and the deepest level
// holds leaves only), so survivors go to the near list alone; a surrogate
// survivor there means a malformed tree and sets DEM_DEV_BAD_TREE.
template <typename T, int N, int BLOCK, bool HALF, bool LEAF = false>
__device__ __forceinline__ void level_batch(const SoupRec<T>* __restrict__ soup, const LevelArgs& a,
                                            LevelShared<BLOCK, LEAF>& sh, uint32_t x, uint32_t first, int n,
                                            LevelCounts& c) {
  constexpr int kR = LevelShared<BLOCK, LEAF>::kRounds;
  const uint32_t bdim = blockDim.x;
  const int4* seg_items = a.qin + (size_t)x * (size_t)a.qcap + first;
  int np = 0, quad_item = 1;
  if ((int)threadIdx.x < n) {
    int4 it = seg_items[threadIdx.x];
    if (it.y < 1 || it.y > DEM_MAX_CHILDREN || it.w < 1 || it.w > DEM_MAX_CHILDREN) {
      atomicOr(a.status, DEM_DEV_BAD_TREE);  // malformed tree: skip the item
      it.y = it.w = 0;
    }
    sh.items[threadIdx.x] = it;
    np = it.y * it.w;
    quad_item = it.y == 4 && it.w == 4;
  }
  // a batch of 4 x 4 products only (the subdivision's children): pair e is
  // child pair e mod 16 of item e / 16, no scan or table needed
  const bool quad = __syncthreads_and(quad_item) != 0;
  int total;
  bool mapped = false;
  if (quad) {
    total = 16 * n;
  } else {
    block_scan(np, sh.offs, sh.wsum, n);
    total = sh.offs[n];
    // small batches map pair -> item through an LDS table; large ones
    // (root chunks) search the offsets
    mapped = total <= BLOCK * 8 && n <= 256;
    if (mapped && (int)threadIdx.x < n) {
      const int o = sh.offs[threadIdx.x];
      for (int q = 0; q < np; ++q) sh.owner[o + q] = (uint8_t)threadIdx.x;
    }
    if (mapped) __syncthreads();
  }
  int round = 0;
  for (int base = 0; base < total; base += bdim, ++round) {
    const int e = base + (int)threadIdx.x;
    bool push_item = false, push_near = false;
    int4 nx = make_int4(0, 0, 0, 0);
    int ci = 0, cj = 0;
    if (e < total) {
      int4 it;
      int qd, rr;
      if (quad) {
        it = sh.items[e >> 4];
        qd = (e >> 2) & 3;
        rr = e & 3;
      } else {
        // item owning flat index e: last k with offs[k] <= e
        int lo = 0, hi = n - 1;
        if (mapped) {
          lo = sh.owner[e];
        } else {
          while (lo < hi) {
            int mid = (lo + hi + 1) >> 1;
            if (sh.offs[mid] <= e) lo = mid; else hi = mid - 1;
          }
        }
        it = sh.items[lo];
        const int l = e - sh.offs[lo];
        const int jn = it.w;
        qd = (int)((float)l * rcp_fast((float)jn));
        rr = l - qd * jn;
        if (rr < 0) { qd -= 1; rr += jn; }
        if (rr >= jn) { qd += 1; rr -= jn; }
      }
      ci = it.x + qd;
      cj = it.z + rr;
      int cbi, cci, pi_, cbj, ccj, pj_;
      bool kfi, kfj;
      Tri<T> A = load_tri(soup, ci, cbi, cci, pi_, kfi);
      Tri<T> B = load_tri(soup, cj, cbj, ccj, pj_, kfj);
      V3<T> D0 = A.v0 - B.v0;
      // what the test needs from the records, formed at once: otherwise the
      // compiler reloads those words after the iteration (an extra L1
      // request per record)
      const T delta = A.eps + B.eps;
      const T slack = bound_slack(A, B, D0, delta);
      T L;
      if constexpr (HALF && sizeof(T) == 4) {
        L = iterate_bound_mixed<N>(A, B, D0, a.ip);
      } else {
        L = iterate_bound<T, N>(A, B, D0, a.ip);
      }
      bool fine = (cci == 0) && (ccj == 0);
      bool keep = a.dense ? true : !(L > delta + slack);
      ++c.evals;
      push_near = keep && fine;
      c.near += push_near;
      if constexpr (LEAF) {
        if (keep && !fine) atomicOr(a.status, DEM_DEV_BAD_TREE);
      } else {
        // surrogate survivors unfold into the next depth's item (only the
        // non-fine side unfolds); fine survivors go to the near list
        push_item = keep && !fine;
        // lazy flattening: a surviving surrogate with fine children has them
        // written before the next depth (plain byte stores of the same value)
        if (a.mark && push_item) {
          if (kfi) a.mark[ci] = 1;
          if (kfj) a.mark[cj] = 1;
        }
        nx.x = cci ? cbi : ci; nx.y = cci ? cci : 1;
        nx.z = ccj ? cbj : cj; nx.w = ccj ? ccj : 1;
        if (push_item && !item_counts_ok(nx)) {
          atomicOr(a.status, DEM_DEV_BAD_TREE);  // malformed tree: drop the item
          push_item = false;
        }
        c.surv += push_item;
      }
    }
    if constexpr (LEAF) {
      lds_append(push_near, make_int2(ci, cj), sh.st.buf, &sh.st.n);
    } else {
      uint32_t slot;
      if (lds_reserve(push_item, &sh.st.ni, slot) && push_item) {
        sh.st.pool[slot] = make_int2(nx.x, nx.z);
        sh.st.cnt[slot] = (uint8_t)(((nx.y - 1) << 4) | (nx.w - 1));
      }
      if (lds_reserve(push_near, &sh.st.nn, slot) && push_near) sh.st.pool[sh.kCap - 1 - slot] = make_int2(ci, cj);
    }
    // check the stages every kR-th round and at the batch's end: after a
    // check at most BLOCK entries remain, kR rounds add at most kR * bdim
    if ((round & (kR - 1)) == kR - 1 || base + (int)bdim >= total) {
      __syncthreads();
      if constexpr (LEAF) {
        if (sh.st.n + kR * bdim > (uint32_t)sh.kCap)
          lds_flush(sh.st, a.near_tail, a.near_, a.ncap, a.status, DEM_DEV_NEAR_OVERFLOW);
      } else {
        // (both lists together: after a check at most BLOCK entries remain)
        if (a.deepest && sh.st.ni != 0u && threadIdx.x == 0) atomicOr(a.status, DEM_DEV_BAD_TREE);
        if (sh.st.ni + sh.st.nn + kR * bdim > (uint32_t)sh.kCap)
          shared_flush(sh.st, a.tail_out, a.qout, a.qcap, a.near_tail, a.near_, a.ncap, a.status);
      }
    }
  }
  __syncthreads();
}

// End of a depth for this block: the staged survivors leave, and the counts
// reach the statistics (block sums into a partial, or one atomic per wave).
template <int BLOCK, bool LEAF>
__device__ __forceinline__ void level_finish(const LevelArgs& a, LevelShared<BLOCK, LEAF>& sh, LevelCounts& c) {
  __syncthreads();
  if constexpr (LEAF) lds_flush(sh.st, a.near_tail, a.near_, a.ncap, a.status, DEM_DEV_NEAR_OVERFLOW);
  else shared_flush(sh.st, a.tail_out, a.qout, a.qcap, a.near_tail, a.near_, a.ncap, a.status);
  if (a.part) {
    unsigned long long v[3] = {c.evals, c.surv, c.near};
    block_sums(v);
    if (threadIdx.x == 0) {
      StatPart& q = a.part[blockIdx.x % kStatPart];
      if (v[0]) atomicAdd(&q.evals[a.depth], v[0]);
      if (v[1]) atomicAdd(&q.survivors[a.depth], v[1]);
      if (v[2]) atomicAdd(&q.near, v[2]);
    }
  } else if (a.stats) {
    unsigned long long s0 = c.evals, s1 = c.surv, s2 = c.near;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      s0 += __shfl_xor(s0, o);
      s1 += __shfl_xor(s1, o);
      s2 += __shfl_xor(s2, o);
    }
    if (lane_id() == 0) {
      if (s0) atomicAdd(&a.stats->evals[a.depth], s0);
      if (s1) atomicAdd(&a.stats->survivors[a.depth], s1);
      if (s2) atomicAdd(&a.stats->near, s2);
    }
  }
  c.evals = c.surv = c.near = 0;
}

// Descent over one tree depth, one launch per depth (Algorithm 5, pairwise
// form).  The blocks of XCD x take the batches of segment x, the items that
// XCD produced at the previous depth (hardware dispatches workgroups
// round-robin over the 8 XCDs, so block b runs on XCD b % 8): a subtree of
// the descent stays on one XCD, whose L2 already holds its triangles.
template <typename T, int N, int BLOCK, bool HALF, bool LEAF = false>
__global__ void __launch_bounds__(BLOCK) k_level(const SoupRec<T>* __restrict__ soup, LevelArgs a) {
  __shared__ LevelShared<BLOCK, LEAF> sh;
  seg_view(sh.view, a.tail_in, a.qcap);
  LevelCounts c{0, 0, 0};
  if (threadIdx.x == 0) stage_reset(sh.st);
  const uint32_t batch = (uint32_t)a.batch;
  const uint32_t x = blockIdx.x % kSeg;
  const uint32_t per = gridDim.x / kSeg + ((blockIdx.x % kSeg) < (gridDim.x % kSeg) ? 1u : 0u);
  const uint32_t fill = sh.view.pre[x + 1] - sh.view.pre[x];
  for (uint32_t first = (blockIdx.x / kSeg) * batch; first < fill; first += per * batch)
    level_batch<T, N, BLOCK, HALF, LEAF>(soup, a, sh, x, first, (int)min(batch, fill - first), c);
  level_finish(a, sh, c);
}

// ------------------------------------------------------------------ persistent descent
// The whole descent of a step in one launch: a grid of co-resident blocks
// seeds the root pairs, then runs every depth with a device work queue --
// each block claims batches of its XCD's segment with one atomic on a
// per-segment claim counter (claimed one batch ahead, so the atomic's latency
// overlaps the current batch) and, once that segment is exhausted, claims
// from the other segments in turn -- followed by the lazy flattening of the
// surviving parents' fine children; grid barriers separate the phases.
// Particle pairs of very different sizes and depths share the grid: a block
// that runs out of its own work takes another XCD's.
//
// The grid barrier waits for every block, so the grid must be co-resident
// (the host sizes it from the occupancy of this kernel).  Each wait is
// bounded: after spin_limit polls the block gives up and sets
// DEM_DEV_STALLED; every block stops at its next barrier once that flag is
// set (a block never runs a phase whose inputs may be incomplete), so the
// kernel always ends, and the host repeats the call with one launch per
// depth.
//
// The barrier is hierarchical, along the XCCs (XCDs): each XCC has its own
// L2, which is not coherent with the others.  A block's stores reach its
// XCC's L2 before it arrives; the last block of an XCC to arrive writes that
// L2 back (one agent-scope release for the XCC, not one per block), arrives
// for the whole XCC, waits for every XCC, invalidates its caches (an
// agent-scope acquire) and releases the XCC's blocks, which then acquire
// too.  A flat barrier (one counter for every block, a release and an
// acquire per block) measured about 110 us per barrier with 1536 blocks;
// this one about 15 us.
constexpr uint32_t kBarrierSpins = 1u << 21;  // polls of ~500 cycles each: about a second

__device__ __forceinline__ uint32_t xcc_id() {
  // HW_REG_XCC_ID (hardware register 20), bits 3:0
  return __builtin_amdgcn_s_getreg((3 << 11) | 20) & (uint32_t)(kMaxXcc - 1);
}

__device__ __forceinline__ uint32_t ld_agent(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Bounded wait until *p >= target (thread 0).  false, with DEM_DEV_STALLED
// set, if the limit is reached or another block has given up.
__device__ __forceinline__ bool wait_at_least(const uint32_t* p, uint32_t target, uint32_t* status,
                                              uint32_t spin_limit) {
  uint32_t spins = 0;
  while (ld_agent(p) < target) {
    if (++spins > spin_limit || (ld_agent(status) & DEM_DEV_STALLED)) {
      atomicOr(status, DEM_DEV_STALLED);
      return false;
    }
    __builtin_amdgcn_s_sleep(8);
  }
  return true;
}

// Thread 0's view of the barrier: its XCC, the blocks resident there, the
// XCCs that hold blocks, the barriers passed.
struct GridBarrier {
  uint32_t x, nx, nact, epoch;
};

// At the kernel's start (thread 0): count this block on its XCC, then arrive
// in its registration group (the group's last block completes the group).
__device__ __forceinline__ void grid_register(Counters* ctr, GridBarrier& b) {
  b.x = xcc_id();
  b.epoch = 0;
  __hip_atomic_fetch_add(&ctr->bar_blocks[b.x][0], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __builtin_amdgcn_s_waitcnt(0);  // the count is performed before the arrival below
  const uint32_t g = blockIdx.x % kSeg;
  const uint32_t gsize = gridDim.x / kSeg + (g < gridDim.x % kSeg ? 1u : 0u);
  if (__hip_atomic_fetch_add(&ctr->bar_reg[g][0], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) + 1u == gsize)
    __hip_atomic_fetch_add(&ctr->bar_reg_top[0], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Every block has registered (thread 0; the grid has at least kSeg blocks):
// read this XCC's block count and the number of XCCs holding blocks.
__device__ __forceinline__ bool grid_ready(Counters* ctr, GridBarrier& b, uint32_t* status, uint32_t spin_limit) {
  if (!wait_at_least(ctr->bar_reg_top, (uint32_t)kSeg, status, spin_limit)) return false;
  b.nx = ld_agent(ctr->bar_blocks[b.x]);
  b.nact = 0;
  for (int x = 0; x < kMaxXcc; ++x) b.nact += ld_agent(ctr->bar_blocks[x]) > 0u;
  return true;
}

// The grid barrier (every thread of every block).  false: the call gave up
// (DEM_DEV_STALLED), the block must stop.
__device__ __forceinline__ bool grid_sync(Counters* ctr, GridBarrier& b, uint32_t* status, uint32_t spin_limit) {
  __shared__ uint32_t s_ok;
  __builtin_amdgcn_s_waitcnt(0);  // this wave's stores have reached the XCC's L2
  __syncthreads();
  if (threadIdx.x == 0) {
    bool ok = !(ld_agent(status) & DEM_DEV_STALLED);
    if (ok) {
      ++b.epoch;
      const uint32_t old = __hip_atomic_fetch_add(&ctr->bar_arrive[b.x][0], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (old + 1u == b.nx * b.epoch) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");  // the XCC's L2 written back
        __hip_atomic_fetch_add(&ctr->bar_top[0], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        ok = wait_at_least(ctr->bar_top, b.nact * b.epoch, status, spin_limit);
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");  // the XCC's L2 and this CU's L1 invalidated
        if (ok) __hip_atomic_store(&ctr->bar_release[b.x][0], b.epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      } else {
        ok = wait_at_least(ctr->bar_release[b.x], b.epoch, status, spin_limit);
        // this compute unit's L1 may hold lines that other blocks have written
        // since: an agent-scope acquire of its own (an L1-only invalidate, at
        // workgroup scope, left stale lines behind)
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      }
    }
    s_ok = ok;
  }
  __syncthreads();
  return s_ok != 0u;
}

// One depth with dynamic claiming.  The first batches of segment x go
// statically to the blocks of x's group (blockIdx % kSeg == x; its r-th
// block takes batch r, no atomic); the rest are claimed with one atomic on
// claim[x] each, one batch ahead so the atomic's latency overlaps the current
// batch.  A block whose segment is exhausted reads the claim counters of the
// segments that have batches beyond their static share (one load each,
// issued together) and claims from the one with the most left, until none
// is left.  A depth's end then costs each block a few loads, not an atomic
// on each of the 8 counters (1536 blocks x 8 atomics on 8 addresses
// serialise for about 100 us).
template <typename T, int N, int BLOCK, bool HALF>
__device__ __forceinline__ void level_dynamic(const SoupRec<T>* __restrict__ soup, const LevelArgs& a,
                                              LevelShared<BLOCK>& sh, uint32_t* claim, LevelCounts& c) {
  seg_view(sh.view, a.tail_in, a.qcap);
  const uint32_t batch = (uint32_t)a.batch;
  const auto group = [](uint32_t y) { return gridDim.x / kSeg + (y < gridDim.x % kSeg ? 1u : 0u); };
  const auto fill = [&](uint32_t y) { return sh.view.pre[y + 1] - sh.view.pre[y]; };
  const auto nbatch = [&](uint32_t y) { return (fill(y) + batch - 1) / batch; };
  uint32_t x = blockIdx.x % kSeg, b = blockIdx.x / kSeg;
  for (;;) {
    if (b < nbatch(x)) {
      __syncthreads();  // every thread has read sh.claim
      if (threadIdx.x == 0)
        sh.claim = nbatch(x) > group(x) ? group(x) + atomicAdd(&claim[x], 1u) : nbatch(x);
      level_batch<T, N, BLOCK, HALF>(soup, a, sh, x, b * batch, (int)min(batch, fill(x) - b * batch), c);
      b = sh.claim;  // level_batch ends with a barrier
      continue;
    }
    __syncthreads();  // every thread has read sh.claim
    if (threadIdx.x == 0) {
      uint32_t taken[kSeg];
#pragma unroll
      for (int y = 0; y < kSeg; ++y) taken[y] = nbatch(y) > group(y) ? ld_agent(&claim[y]) : 0u;
      uint32_t sel = kSeg, most = 0;
#pragma unroll
      for (int y = 0; y < kSeg; ++y) {
        const uint32_t nb = nbatch(y), t = group(y) + taken[y];
        if (nb > t && nb - t > most) { most = nb - t; sel = (uint32_t)y; }
      }
      sh.claim_seg = sel;
      if (sel < kSeg) sh.claim = group(sel) + atomicAdd(&claim[sel], 1u);
    }
    __syncthreads();
    if (sh.claim_seg >= (uint32_t)kSeg) break;
    x = sh.claim_seg;
    b = sh.claim;
  }
}

template <typename T>
struct DescentArgs {
  LevelArgs a;               // near list, statistics, status, iteration, capacities (per-depth fields set here)
  int4* q0;                  // the two level queues
  int4* q1;
  Counters* ctr;
  int n_levels;
  int half_depths;           // depths d < half_depths run the half-precision iteration (FP32 only)
  uint32_t spin_limit;
  int batch[DEM_MAX_LEVELS];
  // seeding
  const int32_t* pairs;
  int n_pairs;
  const int32_t* rbeg;
  const int32_t* rcnt;
  int seed_chunk;
  // lazy flattening (fine_parents null: every record was written by the flatten)
  FlatArgs<T> f;
  const int32_t* fine_parents;
  int fine_parent_begin[DEM_MAX_LEVELS + 1];
};

// 6 waves per SIMD (at most 80 VGPRs), as many as the per-depth kernel gets:
// the phases other than the depth passes (seeding, fine flattening) would
// otherwise raise the register count of the whole kernel.
#ifndef DEM_DESCENT_WAVES
#define DEM_DESCENT_WAVES 6
#endif
template <typename T, int N, int BLOCK, bool HALF>
__global__ void __launch_bounds__(BLOCK, sizeof(T) == 4 ? DEM_DESCENT_WAVES : 1) k_descent(const SoupRec<T>* __restrict__ soup, DescentArgs<T> d) {
  constexpr size_t kL = sizeof(LevelShared<BLOCK>), kF = sizeof(FineShared<T>);
  __shared__ __attribute__((aligned(16))) uint8_t lds[kL > kF ? kL : kF];
  LevelShared<BLOCK>& sh = *reinterpret_cast<LevelShared<BLOCK>*>(lds);
  uint32_t* status = d.a.status;
  GridBarrier bar;
  if (threadIdx.x == 0) grid_register(d.ctr, bar);
  // root pairs of every candidate pair (block-level, pairs in turn)
  for (int pr = blockIdx.x; pr < d.n_pairs; pr += gridDim.x)
    seed_pair(pr, d.pairs, d.n_pairs, d.rbeg, d.rcnt, d.seed_chunk, d.seed_chunk, d.q0, d.ctr->tail[0], d.a.qcap,
              status, sh.claim);
  {
    __shared__ uint32_t s_ready;
    if (threadIdx.x == 0) s_ready = grid_ready(d.ctr, bar, status, d.spin_limit);
    __syncthreads();
    if (!s_ready) return;
  }
  if (!grid_sync(d.ctr, bar, status, d.spin_limit)) return;
  LevelCounts c{0, 0, 0};
  for (int lev = 0; lev < d.n_levels; ++lev) {
    LevelArgs a = d.a;
    a.qin = (lev & 1) ? d.q1 : d.q0;
    a.tail_in = d.ctr->tail[lev];
    a.qout = (lev & 1) ? d.q0 : d.q1;
    a.tail_out = d.ctr->tail[lev + 1];
    a.depth = lev;
    a.deepest = lev == d.n_levels - 1;
    a.batch = d.batch[lev];
    if (threadIdx.x == 0) stage_reset(sh.st);
    if (HALF && lev < d.half_depths)
      level_dynamic<T, N, BLOCK, HALF>(soup, a, sh, d.ctr->claim[lev], c);
    else
      level_dynamic<T, N, BLOCK, false>(soup, a, sh, d.ctr->claim[lev], c);
    level_finish(a, sh, c);
    if (!grid_sync(d.ctr, bar, status, d.spin_limit)) return;
    if (d.fine_parents) {
      const int f0 = d.fine_parent_begin[lev], nf = d.fine_parent_begin[lev + 1] - f0;
      if (nf > 0) {
        fine_range(d.f, d.fine_parents + f0, nf, *reinterpret_cast<FineShared<T>*>(lds), blockIdx.x, gridDim.x);
        if (!grid_sync(d.ctr, bar, status, d.spin_limit)) return;
      }
    }
  }
}

// FLAT: tile = (i range <= blockDim) x (j range <= TJ) of fine triangles.
template <typename T, int N, int TJ>
__global__ void __launch_bounds__(256) k_flat(const SoupRec<T>* __restrict__ soup, LevelArgs a) {
  __shared__ SoupRec<T> tj_s[TJ];
  __shared__ LdsQueue<int2, kStageFlat> qn;
  __shared__ SegView view;
  seg_view(view, a.tail_in, a.qcap);
  const uint32_t count = view.pre[kSeg];
  const uint32_t bdim = blockDim.x;
  unsigned long long my_evals = 0, my_near = 0;
  if (threadIdx.x == 0) qn.n = 0;
  __syncthreads();
  for (uint32_t b = blockIdx.x; b < count; b += gridDim.x) {
    int4 it = a.qin[seg_index(view, b, a.qcap)];
    // stage the j-triangles in LDS
    for (int k = threadIdx.x; k < it.w; k += bdim) tj_s[k] = soup[it.z + k];
    __syncthreads();
    for (int r0 = 0; r0 < it.y; r0 += bdim) {
      const int r = r0 + (int)threadIdx.x;
      const bool act = r < it.y;
      const int ci = it.x + (act ? r : 0);
      int cbi, cci, pi_;
      Tri<T> A = load_tri(soup, ci, cbi, cci, pi_);
      for (int k = 0; k < it.w; ++k) {
        int cbj, ccj, pj_;
        Tri<T> B = load_tri(tj_s, k, cbj, ccj, pj_);
        V3<T> D0 = A.v0 - B.v0;
        T L = iterate_bound<T, N>(A, B, D0, a.ip);
        T delta = A.eps + B.eps;
        bool keep = act && (a.dense ? true : !(L > delta + bound_slack(A, B, D0, delta)));
        my_evals += act;
        my_near += keep;
        lds_append(keep, make_int2(ci, it.z + k), qn.buf, &qn.n);
        if (k % 4 == 3 || k == it.w - 1) {
          // at most 4 * bdim appends since the last check
          __syncthreads();
          if (qn.n + 4 * bdim > (uint32_t)kStageFlat)
            lds_flush(qn, a.near_tail, a.near_, a.ncap, a.status, DEM_DEV_NEAR_OVERFLOW);
        }
      }
    }
    __syncthreads();
  }
  lds_flush(qn, a.near_tail, a.near_, a.ncap, a.status, DEM_DEV_NEAR_OVERFLOW);
  if (a.stats) {
    unsigned long long s0 = my_evals, s2 = my_near;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      s0 += __shfl_xor(s0, o);
      s2 += __shfl_xor(s2, o);
    }
    if (lane_id() == 0) {
      if (s0) atomicAdd(&a.stats->evals[0], s0);
      if (s2) atomicAdd(&a.stats->near, s2);
    }
  }
}

struct NearArgs {
  const int2* near_;       // pairs to settle
  const uint32_t* near_tail;
  int64_t ncap;
  int2* fb;                // certify pass: pairs left for the exact pass
  uint32_t* fb_tail;
  int32_t* pi;
  int32_t* pj;
  int32_t* ti;
  int32_t* tj;
  void* d;
  void* x;
  void* n;
  uint32_t* count;
  int64_t ccap;
  int dense;
  double k;
  double* energy;
  dem_stats* stats;
  uint32_t* status;
  IterParams ip;
  // frontier step: list entries are leaf indices; the leaves live in
  // fr_buf[fr_state[0]] and each settled leaf's outcome byte is written
  const int4* fr_buf0;
  const int4* fr_buf1;
  const uint32_t* fr_state;
  uint8_t* fr_meta;
  void* adj;               // contacts' adjoint rows, or null
  StatPart* part;          // partial statistics and energy (null: straight into stats / energy)
};

// A contact on its way out: its output fields and its adjoint rows.
template <typename T>
struct ContactRec {
  int32_t pi, pj, ti, tj;
  T d, x[3], n[3];
  T adj[DEM_ADJOINT_ROWS];
};

// Contacts staged in LDS field by field (one array per field), so that the
// lanes appending consecutive slots, and the threads copying them out, touch
// consecutive words (an array of 80-byte records put consecutive lanes 20
// words apart: conflicting banks on every access).
constexpr int kContactFields = 7 + DEM_ADJOINT_ROWS;  // d, x[3], n[3], adjoint rows
template <typename T, int CAP>
struct ContactStage {
  int32_t id[4][CAP];        // pi, pj, ti, tj
  T f[kContactFields][CAP];
  uint32_t n;
  uint32_t gbase;
};

// 496 FP32 records (80 bytes) keep a block of the exact pass within 40 KB of
// LDS: four blocks per CU, as many as its registers allow.
constexpr int kStageContacts = 496;

// Adjoint rows of a settled pair (the layout is described with dem_contacts).
template <typename T>
__device__ __forceinline__ void adjoint_rows(T adj[DEM_ADJOINT_ROWS], T delta, T d, V3<T> cp, V3<T> cq,
                                             const BaryCode<T>& kp, const BaryCode<T>& kq) {
  const V3<T> u = d > T(0) ? (T(1) / d) * (cq - cp) : V3<T>{T(0), T(0), T(0)};
  adj[0] = delta;
  adj[1] = u.x; adj[2] = u.y; adj[3] = u.z;
  adj[4] = T(kp.code + 8 * kq.code);
  adj[5] = kp.a; adj[6] = kp.b;
  adj[7] = kq.a; adj[8] = kq.b;
}

// Wave-aggregated append of rec (lanes with pred) to the stage.
template <typename T, int CAP>
__device__ __forceinline__ void stage_contact(bool pred, const ContactRec<T>& rec, ContactStage<T, CAP>& qc) {
  unsigned long long m = __ballot(pred);
  if (m == 0ull) return;
  int leader = __ffsll((long long)m) - 1;
  uint32_t base = 0;
  if (lane_id() == leader) base = atomicAdd(&qc.n, (uint32_t)__popcll(m));
  base = (uint32_t)__builtin_amdgcn_readlane((int)base, leader);
  unsigned long long lt = (lane_id() == 0) ? 0ull : (~0ull >> (64 - lane_id()));
  if (pred) {
    const uint32_t k = base + (uint32_t)__popcll(m & lt);
    qc.id[0][k] = rec.pi; qc.id[1][k] = rec.pj; qc.id[2][k] = rec.ti; qc.id[3][k] = rec.tj;
    qc.f[0][k] = rec.d;
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      qc.f[1 + q][k] = rec.x[q];
      qc.f[4 + q][k] = rec.n[q];
    }
#pragma unroll
    for (int q = 0; q < DEM_ADJOINT_ROWS; ++q) qc.f[7 + q][k] = rec.adj[q];
  }
}

template <typename T>
__device__ __forceinline__ void write_contacts(ContactStage<T, kStageContacts>& qc, const NearArgs& a) {
  T* dd = static_cast<T*>(a.d);
  T* xx = static_cast<T*>(a.x);
  T* nn = static_cast<T*>(a.n);
  T* aj = static_cast<T*>(a.adj);
  if (threadIdx.x == 0) qc.gbase = qc.n ? atomicAdd(a.count, qc.n) : 0u;
  __syncthreads();
  for (uint32_t k = threadIdx.x; k < qc.n; k += blockDim.x) {
    uint64_t slot = (uint64_t)qc.gbase + k;
    if (slot < (uint64_t)a.ccap) {
      a.pi[slot] = qc.id[0][k]; a.pj[slot] = qc.id[1][k]; a.ti[slot] = qc.id[2][k]; a.tj[slot] = qc.id[3][k];
      dd[slot] = qc.f[0][k];
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        xx[q * a.ccap + slot] = qc.f[1 + q][k];
        nn[q * a.ccap + slot] = qc.f[4 + q][k];
      }
      if (aj) {
#pragma unroll
        for (int q = 0; q < DEM_ADJOINT_ROWS; ++q) aj[q * a.ccap + slot] = qc.f[7 + q][k];
      }
    } else {
      atomicOr(a.status, DEM_DEV_CONTACT_OVERFLOW);
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) qc.n = 0;
  __syncthreads();
}

// Certification tolerances (FP32 / FP64): accept U when U - L* <= rel U + abs,
// abs proportional to the pair's size bounds.
template <typename T>
struct CertTol;
template <>
struct CertTol<float> {
  static constexpr float rel = 4e-6f, abs = 1e-7f;
};
template <>
struct CertTol<double> {
  static constexpr double rel = 1e-13, abs = 1e-15;
};

// Settle near pairs (fine pairs the lower bound did not prune) and emit the
// contacts, d <= eps_i + eps_j.  CERTIFY: the iterate + snap + certificate
// of certify_pair(); pairs it cannot settle go to the fallback list.
// Otherwise: the exact comparison-based distance for every listed pair.
// FR: entries are frontier leaf indices (see k_fr_eval); the leaf's outcome
// becomes "contact" or "no contact".
// (FP32: at most 128 VGPRs, four waves per SIMD, which the staging LDS
// also allows)
template <typename T, int N, bool CERTIFY, bool FR>
__global__ void __launch_bounds__(256, sizeof(T) == 4 ? 4 : 1) k_near(const SoupRec<T>* __restrict__ soup, NearArgs a) {
  __shared__ ContactStage<T, kStageContacts> qc;
  __shared__ LdsQueue<int2, kStageNear> qf;
  __shared__ SegView view;
  seg_view(view, a.near_tail, a.ncap);
  const uint32_t bdim = blockDim.x;
  double e_acc = 0.0;
  unsigned long long my_fb = 0, my_cert = 0, my_c = 0;
  if (threadIdx.x == 0) { qc.n = 0; qf.n = 0; }
  __syncthreads();
  // the blocks of XCD x (b % 8 == x) take segment x: the near pairs that XCD
  // found at the last depth, whose triangles its L2 may still hold
  const uint32_t x = blockIdx.x % kSeg;
  const uint32_t per = gridDim.x / kSeg + ((blockIdx.x % kSeg) < (gridDim.x % kSeg) ? 1u : 0u);
  const uint32_t fill = view.pre[x + 1] - view.pre[x];
  const int2* seg = a.near_ + (size_t)x * (size_t)a.ncap;
  for (uint32_t base = (blockIdx.x / kSeg) * bdim; base < fill; base += per * bdim) {
    const uint32_t e = base + threadIdx.x;
    bool emit = false, defer = false;
    ContactRec<T> rec;
    int2 pr = make_int2(0, 0);
    if (e < fill) {
      pr = seg[e];
      int ta = pr.x, tb = pr.y;
      if constexpr (FR) {
        const int4 lf = (a.fr_state[0] ? a.fr_buf1 : a.fr_buf0)[pr.x];
        ta = lf.x;
        tb = lf.y;
      }
      int cbi, cci, cbj, ccj, pi_, pj_;
      Tri<T> A = load_tri(soup, ta, cbi, cci, pi_);
      Tri<T> B = load_tri(soup, tb, cbj, ccj, pj_);
      V3<T> D0 = A.v0 - B.v0;
      T d;
      V3<T> cp, cq;
      BaryCode<T> kp, kq;
      bool settled = true;
      if constexpr (CERTIFY) {
        T wp[3], wq[3];
        settled = certify_pair<T, N>(A, B, D0, a.ip, CertTol<T>::rel, CertTol<T>::abs * (A.size + B.size),
                                     d, cp, cq, wp, wq, kp, kq);
        my_cert += settled;
        defer = !settled;
      } else {
        Closest<T> c;
        exact_tri_tri(V3<T>{0, 0, 0}, A.e1, A.e2, -D0, B.e1, B.e2, c);
        ++my_fb;
        d = sq_(c.d2);
        cp = c.p;
        cq = c.q;
        kp = c.cp;
        kq = c.cq;
      }
      if (settled) {
        T delta = a.dense ? T(INFINITY) : A.eps + B.eps;
        emit = d <= delta;
        if (!isfinite(d)) atomicOr(a.status, DEM_DEV_NONFINITE);
        // contact point at the centre of the overlap of the two environments
        V3<T> w = cq - cp;
        T lam = d > T(0) ? (d + A.eps - B.eps) / (T(2) * d) : T(0);
        V3<T> xl = fma3(lam, w, cp);
        V3<T> nc = cp - xl;
        V3<T> xc = xl + A.v0;
        rec.pi = pi_; rec.pj = pj_; rec.ti = ta; rec.tj = tb; rec.d = d;
        if constexpr (FR) a.fr_meta[4 * (size_t)pr.x] = (uint8_t)(emit ? kOutKeep : kOutPrune);
        rec.x[0] = xc.x; rec.x[1] = xc.y; rec.x[2] = xc.z;
        rec.n[0] = nc.x; rec.n[1] = nc.y; rec.n[2] = nc.z;
        adjoint_rows(rec.adj, A.eps + B.eps, d, cp, cq, kp, kq);
        if (emit && !a.dense) {
          double pen = (double)delta - (double)d;
          e_acc += a.k * pen * pen;
        }
        my_c += emit;
      }
    }
    stage_contact(emit, rec, qc);
    if constexpr (CERTIFY) lds_append(defer, pr, qf.buf, &qf.n);
    __syncthreads();
    if (qc.n + bdim > (uint32_t)kStageContacts) write_contacts(qc, a);
    if constexpr (CERTIFY) {
      if (qf.n + bdim > (uint32_t)kStageNear)
        lds_flush(qf, a.fb_tail, a.fb, a.ncap, a.status, DEM_DEV_NEAR_OVERFLOW);
    }
  }
  write_contacts(qc, a);
  if constexpr (CERTIFY) lds_flush(qf, a.fb_tail, a.fb, a.ncap, a.status, DEM_DEV_NEAR_OVERFLOW);
  if (a.part) {
    // block sums into this block's partial (k_fold_stats adds them up)
    unsigned long long v[3] = {my_fb, my_c, my_cert};
    block_sums(v);
    const double esum = a.energy ? block_sum_f64(e_acc) : 0.0;
    if (threadIdx.x == 0) {
      StatPart& q = a.part[blockIdx.x % kStatPart];
      if (a.stats) {
        if (v[0]) atomicAdd(&q.fallback, v[0]);
        if (v[1]) atomicAdd(&q.contacts, v[1]);
        if (v[2]) atomicAdd(&q.certified, v[2]);
      }
      if (esum != 0.0) atomicAdd(&q.energy, esum);
    }
    return;
  }
  if (a.energy) {
    double sum = wave_sum(e_acc);
    if (lane_id() == 0 && sum != 0.0) atomicAdd(a.energy, sum);
  }
  if (a.stats) {
    unsigned long long s0 = my_fb, s1 = my_c, s2 = my_cert;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      s0 += __shfl_xor(s0, o);
      s1 += __shfl_xor(s1, o);
      s2 += __shfl_xor(s2, o);
    }
    if (lane_id() == 0) {
      if (s0) atomicAdd(&a.stats->fallback, s0);
      if (s1) atomicAdd(&a.stats->contacts, s1);
      if (s2) atomicAdd(&a.stats->certified, s2);
    }
  }
}

template <typename T>
__device__ __forceinline__ void atomic_add_t(T* p, T v) {
  unsafeAtomicAdd(p, v);
}

// Gradient accumulation in LDS: contributions of a chunk of contacts are
// summed per vertex in an open-addressing hash table before one global
// atomic per (vertex, component) leaves the block.  Contacts arrive grouped
// by the surrogate pair they descend from, so a chunk touches few distinct
// vertices (about 0.43 per contact in the 1000-sphere lattice); scattered
// device-scope float atomics are the costly part.
// A thread takes kBwdPerThread consecutive contacts.  The child pairs of a
// surrogate pair are listed with the triangle of particle i varying slowest,
// so consecutive contacts often share t_i: the contributions of such a run
// to the vertices of t_i are summed in registers and enter the table once.
//
// The table sums in 64-bit fixed point: LDS float atomics are executed far
// slower than integer ones on this GPU (measured: about 190 CU cycles per
// wave-wide ds_add_f32, whatever the addresses, against about 5 for
// ds_add_u32 on distinct banks).  Every contribution of a chunk is bounded
// by B = 2 k |dE| max delta (the penetration is at most delta, weights and
// the components of the unit direction at most 1), and a value entering the
// table sums at most four of them (a run of t_i, or a quad's merged t_j).
// With B < 2^e a value c enters as round(c 2^(F - e)): F = 28 in FP32 (a
// 32-bit conversion, |c 2^(F-e)| < 2^30; error at most 2^-29 B, below the
// FP32 rounding of any contribution above B / 32), F = 51 in FP64.  A slot
// takes at most two contributions per contact of the chunk (2^11), so the
// 64-bit sums cannot overflow, and they are exact: the one rounding on the
// way out is that of the conversion back to T.  A contribution above 2^100
// (or not finite) has no place in them: it sets DEM_DEV_NONFINITE and is
// left out.
constexpr int kHashSlots = 1024;     // power of two
constexpr int kHashBits = 10;
constexpr int kBwdPerThread = 4;     // consecutive contacts per thread per chunk

template <typename T>
struct GradHash {
  int key[kHashSlots];
  unsigned long long val[3][kHashSlots];
  uint32_t dmax;   // FP32 bits of the chunk's largest delta (rounded up)
};

// Home slot of vertex vid: its low bits, xor-ed with a multiple of its
// 1024-wide id window (so that windows of different particles spread).
// Vertices of a contact patch have nearby ids, so neighbouring slots hold
// neighbouring vertices, and the lanes of a flush instruction add to the
// same cache lines of the gradient: the device-scope atomics leave in far
// fewer memory requests than from a scattering hash (measured: the backward
// of the 1000-sphere lattice 0.316 -> 0.232 ms).
__device__ __forceinline__ uint32_t hash_slot(int vid) {
  return ((uint32_t)vid ^ ((uint32_t)vid >> kHashBits) * 0x9E5u) & (kHashSlots - 1);
}

template <typename T>
struct FixedPoint;
template <>
struct FixedPoint<float> {
  static constexpr int F = 28;
  static __device__ __forceinline__ unsigned long long to(float c, float s) {
    return (unsigned long long)(long long)__float2int_rn(c * s);
  }
};
template <>
struct FixedPoint<double> {
  static constexpr int F = 51;
  static __device__ __forceinline__ unsigned long long to(double c, double s) {
    return (unsigned long long)__double2ll_rn(c * s);
  }
};

// Scale 2^(F - e) and its inverse for a chunk whose contributions are at
// most B (B < 2^e; exponents kept inside the FP32 range).
template <typename T>
__device__ __forceinline__ void fixed_scale(double B, T& s, T& inv) {
  int e = 0;
  if (B > 0.0) (void)frexp(B, &e);
  e = max(-60, min(e, 102));
  s = (T)ldexp(1.0, FixedPoint<T>::F - e);
  inv = (T)ldexp(1.0, e - FixedPoint<T>::F);
}

template <typename T>
__device__ __forceinline__ void hash_add(GradHash<T>& H, int vid, T gx, T gy, T gz, T s, T* grad,
                                         int n_verts) {
  uint32_t h = hash_slot(vid);
#pragma unroll 1
  for (int probe = 0; probe < 32; ++probe) {
    int cur = atomicCAS(&H.key[h], -1, vid);
    if (cur == -1 || cur == vid) {
      atomicAdd(&H.val[0][h], FixedPoint<T>::to(gx, s));
      atomicAdd(&H.val[1][h], FixedPoint<T>::to(gy, s));
      atomicAdd(&H.val[2][h], FixedPoint<T>::to(gz, s));
      return;
    }
    h = (h + 1) & (kHashSlots - 1);
  }
  unsafeAtomicAdd(grad + vid, gx);  // crowded table: straight to memory
  unsafeAtomicAdd(grad + n_verts + vid, gy);
  unsafeAtomicAdd(grad + 2 * (size_t)n_verts + vid, gz);
}

// The three vertex contributions of triangle t (gv[v] for vertex v): index
// loads and first probes are issued together so their latencies overlap.
template <typename T>
__device__ __forceinline__ void hash_add_tri(GradHash<T>& H, const int32_t* __restrict__ tv, int n_tris,
                                             int t, const V3<T>* gv, T s, T* grad, int n_verts) {
  int vid[3], slot[3], cur[3];
#pragma unroll
  for (int v = 0; v < 3; ++v) vid[v] = tv[(size_t)v * n_tris + t];
#pragma unroll
  for (int v = 0; v < 3; ++v) {
    const bool nz = gv[v].x != T(0) || gv[v].y != T(0) || gv[v].z != T(0);
    slot[v] = (int)hash_slot(vid[v]);
    // a plain read first: most vertices of a chunk are already in the table,
    // and only an empty slot needs the compare-and-swap
    cur[v] = nz ? H.key[slot[v]] : -2;
  }
#pragma unroll
  for (int v = 0; v < 3; ++v)
    if (cur[v] == -1) cur[v] = atomicCAS(&H.key[slot[v]], -1, vid[v]);
#pragma unroll
  for (int v = 0; v < 3; ++v) {
    if (cur[v] == -2) continue;
    if (cur[v] == -1 || cur[v] == vid[v]) {
      atomicAdd(&H.val[0][slot[v]], FixedPoint<T>::to(gv[v].x, s));
      atomicAdd(&H.val[1][slot[v]], FixedPoint<T>::to(gv[v].y, s));
      atomicAdd(&H.val[2][slot[v]], FixedPoint<T>::to(gv[v].z, s));
    } else {
      hash_add(H, vid[v], gv[v].x, gv[v].y, gv[v].z, s, grad, n_verts);  // probe on
    }
  }
}

// Lanes of a quad exchange values with DPP quad permutations (VALU moves, no
// LDS): QUAD_XOR1 swaps lanes 2k and 2k+1, QUAD_XOR2 lanes k and k^2.
constexpr int kQuadXor1 = 0xB1;  // quad_perm [1, 0, 3, 2]
constexpr int kQuadXor2 = 0x4E;  // quad_perm [2, 3, 0, 1]

template <int CTRL>
__device__ __forceinline__ int quad_swap(int v) {
  return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, false);
}
template <int CTRL>
__device__ __forceinline__ float quad_swap(float v) {
  return __int_as_float(quad_swap<CTRL>(__float_as_int(v)));
}
template <int CTRL>
__device__ __forceinline__ double quad_swap(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = quad_swap<CTRL>((int)(b & 0xFFFFFFFFll)), hi = quad_swap<CTRL>((int)(b >> 32));
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// One step of the quad merge: a lane whose partner holds the same key adds
// the partner's contribution (the lower lane) or gives its own away (the
// upper lane, whose key becomes unique and negative).  Every lane of the
// wave must take part.
template <int CTRL, int M, typename T>
__device__ __forceinline__ void quad_merge_step(int& key, V3<T> (&g)[3]) {
  const int pk = quad_swap<CTRL>(key);
  V3<T> pg[3];
#pragma unroll
  for (int v = 0; v < 3; ++v) pg[v] = V3<T>{quad_swap<CTRL>(g[v].x), quad_swap<CTRL>(g[v].y), quad_swap<CTRL>(g[v].z)};
  const bool same = pk == key;
  const bool lower = (lane_id() & M) == 0;
#pragma unroll
  for (int v = 0; v < 3; ++v) g[v] = (same && lower) ? g[v] + pg[v] : g[v];
  key = (same && !lower) ? -2 - lane_id() : key;
}

// Four consecutive values with 16-byte loads (p 16-byte aligned).
__device__ __forceinline__ void ld4(const int32_t* p, int32_t o[4]) {
  const int4 v = *reinterpret_cast<const int4*>(p);
  o[0] = v.x; o[1] = v.y; o[2] = v.z; o[3] = v.w;
}
__device__ __forceinline__ void ld4(const float* p, float o[4]) {
  const float4 v = *reinterpret_cast<const float4*>(p);
  o[0] = v.x; o[1] = v.y; o[2] = v.z; o[3] = v.w;
}
__device__ __forceinline__ void ld4(const double* p, double o[4]) {
  const double2 a = reinterpret_cast<const double2*>(p)[0], b = reinterpret_cast<const double2*>(p)[1];
  o[0] = a.x; o[1] = a.y; o[2] = b.x; o[3] = b.y;
}

// ADJ: d from the contacts and delta, u and the weights from their adjoint
// rows (no triangle data read); with VEC (rows 16-byte aligned, capacity a
// multiple of 4, so the four entries from a multiple of 4 below the count
// are inside the arrays) a thread reads its four contacts' fields with one
// 16-byte load per row.  Otherwise the pair's closest points are solved
// again from the soup records.
template <typename T, bool ADJ, bool VEC>
__global__ void __launch_bounds__(256, sizeof(T) == 4 ? 4 : 1) k_backward(const SoupRec<T>* __restrict__ soup,
                                                  const int32_t* __restrict__ tv, int n_tris,
                                                  int n_verts, const int32_t* __restrict__ cti,
                                                  const int32_t* __restrict__ ctj, const T* __restrict__ cd,
                                                  const T* __restrict__ adj,
                                                  const uint32_t* __restrict__ ccount, int64_t ccap,
                                                  double k, const double* __restrict__ grad_E,
                                                  T* __restrict__ grad, double* energy,
                                                  uint32_t* status) {
  static_assert(kBwdPerThread == 4, "the vector reads take four contacts");
  __shared__ GradHash<T> H;
  const uint32_t cnt = min((uint64_t)*ccount, (uint64_t)ccap);
  const double gE = grad_E ? *grad_E : 1.0;
  const uint32_t bdim = blockDim.x;
  const uint32_t chunk = bdim * kBwdPerThread;
  for (int s2 = threadIdx.x; s2 < kHashSlots; s2 += bdim) {
    H.key[s2] = -1;
    H.val[0][s2] = H.val[1][s2] = H.val[2][s2] = 0ull;
  }
  if (threadIdx.x == 0) H.dmax = 0u;
  __syncthreads();
  const double g_bound = 2.0 * k * fabs(gE);  // times delta: a contribution's bound
  double e_acc = 0.0;
  for (uint32_t c0 = blockIdx.x * chunk; c0 < cnt; c0 += gridDim.x * chunk) {
    const uint32_t cb = c0 + threadIdx.x * kBwdPerThread;
    int run = -1;      // t_i of the current run
    V3<T> rg[3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};  // its vertex contributions so far
    int pti[kBwdPerThread], ptj[kBwdPerThread];
    T pd[kBwdPerThread], pa[DEM_ADJOINT_ROWS][kBwdPerThread];
    if constexpr (ADJ) {
      const size_t C = (size_t)ccap;
      if constexpr (VEC) {
        ld4(cti + cb, pti);
        ld4(ctj + cb, ptj);
        ld4(cd + cb, pd);
#pragma unroll
        for (int q = 0; q < DEM_ADJOINT_ROWS; ++q) ld4(adj + q * C + cb, pa[q]);
      } else {
#pragma unroll
        for (int j = 0; j < kBwdPerThread; ++j) {
          const uint32_t c = min(cb + j, cnt - 1);  // (entries past cnt are not used)
          pti[j] = cti[c];
          ptj[j] = ctj[c];
          pd[j] = cd[c];
#pragma unroll
          for (int q = 0; q < DEM_ADJOINT_ROWS; ++q) pa[q][j] = adj[q * C + c];
        }
      }
    }
    // the chunk's largest delta (of contacts within the count), for the
    // fixed-point scale of its table
    {
      float dm = 0.0f;
#pragma unroll
      for (int j = 0; j < kBwdPerThread; ++j) {
        const uint32_t c = cb + j;
        if (c >= cnt) continue;
        T dl;
        if constexpr (ADJ) {
          dl = pa[0][j];
        } else {
          const int ti = cti[c], tj = ctj[c];
          dl = ((uint32_t)ti < (uint32_t)n_tris && (uint32_t)tj < (uint32_t)n_tris)
                   ? soup[ti].g[3] + soup[tj].g[3] : T(0);
        }
        // (FP64: rounded up to FP32 so that it stays a bound)
        const float df = sizeof(T) == 8 ? __double2float_ru((double)dl) : (float)dl;
        if (df > dm && df <= 3.0e38f) dm = df;  // (non-finite deltas give no contribution)
      }
      uint32_t b = __float_as_uint(dm);
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) b = max(b, (uint32_t)__shfl_xor((int)b, o));
      if (lane_id() == 0 && b) atomicMax(&H.dmax, b);
    }
    __syncthreads();
    T fs, finv;
    fixed_scale<T>(g_bound * (double)__uint_as_float(H.dmax), fs, finv);
    // The contacts of a thread's step j and of the next lanes' step j are four
    // apart in the list: in a surrogate pair's 4 x 4 children they share t_j.
    // So at each step the four lanes of a quad merge equal t_j with DPP
    // swaps, and one lane per distinct t_j enters the table.  (Flags instead
    // of early exits keep every lane in step for the swaps.)
#pragma unroll
    for (int j = 0; j < kBwdPerThread; ++j) {
      const uint32_t c = cb + j;
      bool live = c < cnt;
      const uint32_t cr = live ? c : cnt - 1;
      const int ti = ADJ ? pti[j] : cti[cr], tj = ADJ ? ptj[j] : ctj[cr];
      if (live && ((uint32_t)ti >= (uint32_t)n_tris || (uint32_t)tj >= (uint32_t)n_tris)) {
        atomicOr(status, DEM_DEV_BAD_TREE);  // not a triangle of this scene: skipped
        live = false;
      }
      T d = T(0), delta = T(-1), wp[3] = {T(0), T(0), T(0)}, wq[3] = {T(0), T(0), T(0)};
      V3<T> u = {T(0), T(0), T(0)};
      if (live) {
        if constexpr (ADJ) {
          d = pd[j];
          delta = pa[0][j];
          u = V3<T>{pa[1][j], pa[2][j], pa[3][j]};
          const int code = (int)pa[4][j];
          bary_weights(code & 7, pa[5][j], pa[6][j], wp);
          bary_weights(code >> 3, pa[7][j], pa[8][j], wq);
        } else {
          int cbi, cci, pi_, cbj, ccj, pj_;
          Tri<T> A = load_tri(soup, ti, cbi, cci, pi_);
          Tri<T> B = load_tri(soup, tj, cbj, ccj, pj_);
          V3<T> D0 = A.v0 - B.v0;
          Closest<T> cl;
          exact_tri_tri(V3<T>{0, 0, 0}, A.e1, A.e2, -D0, B.e1, B.e2, cl);
          d = sq_(cl.d2);
          delta = A.eps + B.eps;
          u = d > T(0) ? (T(1) / d) * (cl.q - cl.p) : V3<T>{T(0), T(0), T(0)};
#pragma unroll
          for (int v = 0; v < 3; ++v) {
            wp[v] = cl.wp[v];
            wq[v] = cl.wq[v];
          }
        }
      }
      const double pen = (double)delta - (double)d;
      live = live && pen >= 0.0;
      if (live) e_acc += k * pen * pen;
      bool on = live && d > T(0) && grad != nullptr;
      T g = on ? T(2.0 * k * pen * gE) : T(0);
      if (on && !(fabs((double)g) <= 0x1p100)) {  // no place in the fixed-point sums
        atomicOr(status, DEM_DEV_NONFINITE);
        on = false;
        g = T(0);
      }
      if (on) {
        if (ti != run) {
          if (run >= 0) hash_add_tri(H, tv, n_tris, run, rg, fs, grad, n_verts);
          run = ti;
#pragma unroll
          for (int v = 0; v < 3; ++v) rg[v] = V3<T>{0, 0, 0};
        }
#pragma unroll
        for (int v = 0; v < 3; ++v) rg[v] = rg[v] + (g * wp[v]) * u;
      }
      V3<T> gq[3];
#pragma unroll
      for (int v = 0; v < 3; ++v) gq[v] = (-g * wq[v]) * u;
      int key = on ? tj : -2 - lane_id();
      quad_merge_step<kQuadXor1, 1>(key, gq);
      quad_merge_step<kQuadXor2, 2>(key, gq);
      if (key >= 0) hash_add_tri(H, tv, n_tris, key, gq, fs, grad, n_verts);
    }
    if (run >= 0) hash_add_tri(H, tv, n_tris, run, rg, fs, grad, n_verts);
    __syncthreads();
    for (int s2 = threadIdx.x; s2 < kHashSlots; s2 += bdim) {
      int vid = H.key[s2];
      if (vid >= 0) {
        unsafeAtomicAdd(grad + vid, (T)(long long)H.val[0][s2] * finv);
        unsafeAtomicAdd(grad + n_verts + vid, (T)(long long)H.val[1][s2] * finv);
        unsafeAtomicAdd(grad + 2 * (size_t)n_verts + vid, (T)(long long)H.val[2][s2] * finv);
        H.key[s2] = -1;
        H.val[0][s2] = H.val[1][s2] = H.val[2][s2] = 0ull;
      }
    }
    if (threadIdx.x == 0) H.dmax = 0u;
    __syncthreads();
  }
  if (energy) {
    double sum = wave_sum(e_acc);
    if (lane_id() == 0 && sum != 0.0) atomicAdd(energy, sum);
  }
}

// ------------------------------------------------------------------ frontier
// Persistent active sets (Section 5.3, Algorithm 6 in pairwise form; the
// leaf record and buffer layout are described with dem_frontier in dem.h).
//
// One dem_frontier_step:
//   k_fr_eval   every leaf (blocks take contiguous ranges, fr_range): in
//               range or not (lower bound, or exact distance); fine pairs in
//               range go to the near list; per-leaf outcome word (meta) =
//               outcome | group index << 8 | n << 16 with n = the group size
//               at a group's first leaf that may narrow, or the child-pair
//               count of a leaf that widens; per-block output leaf counts
//   k_near<FR>  exact distance of the fine pairs, contacts, outcome byte
//   k_fr_group  a group's first leaf checks that its n members follow it in
//               order, all leaves and all "no contact"; marks them (cm) and
//               takes the removed members off their blocks' counts
//   k_fr_scan   block offsets (one block)
//   k_fr_emit   rewrite in depth-first order into the other buffer: copies,
//               parents of narrowed groups (inserted into the memory set),
//               child pairs of widened leaves (memory set looked up)
//   k_fr_finish switch buffers when something changed
constexpr unsigned long long kMemEmpty = ~0ull;
constexpr int kScanThreads = 1024;
constexpr int kFrBlock = 256;
constexpr int kMemProbes = 64;
constexpr int kFrMaxGrid = 8192;  // blocks of the per-leaf kernels (scan partials)

__device__ __forceinline__ uint32_t fr_depth(uint32_t info) { return (info >> 17) & 31u; }
__device__ __forceinline__ uint32_t fr_gidx(uint32_t info) { return info & 255u; }
__device__ __forceinline__ uint32_t fr_gsize(uint32_t info) { return (info >> 8) & 511u; }
__device__ __forceinline__ uint32_t fr_info(uint32_t g, uint32_t n, uint32_t D, uint32_t si, uint32_t sj) {
  return g | (n << 8) | (D << 17) | (si << 22) | (sj << 23);
}

struct FrontierArgs {
  int4* buf0;
  int4* buf1;
  uint32_t* state;              // {current buffer, leaf count, leaves needed, 0}
  int64_t cap;
  unsigned long long* mem;      // memory set (open addressing)
  uint64_t mem_mask;
  uint32_t* meta;               // [cap] per-leaf outcome word
  uint8_t* cm;                  // [cap] narrowing marks: 2 = group's first leaf, 1 = other member
  unsigned long long* part;     // [grid + 1] output leaves per block -> offsets
  StatPart* spart;              // partial statistics (null: straight into stats)
  const int32_t* tri_parent;
  const uint8_t* tri_depth;
  const int32_t* cbeg;
  const int32_t* ccnt;
  int n_tris;
  Counters* ctr;
  int2* near_;
  uint32_t* near_tail;
  int64_t ncap;
  dem_stats* stats;
  uint32_t* status;
  IterParams ip;
};

__device__ __forceinline__ uint32_t fr_count(const FrontierArgs& a) {
  return (uint32_t)min((uint64_t)a.state[1], (uint64_t)a.cap);
}

__device__ __forceinline__ unsigned long long mem_key(int ta, int tb) {
  return ((unsigned long long)(uint32_t)ta << 32) | (uint32_t)tb;
}

__device__ __forceinline__ uint64_t mem_slot(unsigned long long key, uint64_t mask) {
  return (uint64_t)((key * 0x9E3779B97F4A7C15ull) >> 29) & mask;
}

// Slots are never cleared within a run of steps, so a probe chain up to a
// stored key holds no empty slot: a lookup may stop at the first empty one.
__device__ bool mem_contains(const FrontierArgs& a, unsigned long long key) {
  uint64_t h = mem_slot(key, a.mem_mask);
  for (int k = 0; k < kMemProbes; ++k) {
    const unsigned long long v = a.mem[h];
    if (v == key) return true;
    if (v == kMemEmpty) return false;
    h = (h + 1) & a.mem_mask;
  }
  atomicOr(a.status, DEM_DEV_FRONTIER_OVERFLOW);
  return false;
}

__device__ void mem_insert(const FrontierArgs& a, unsigned long long key) {
  uint64_t h = mem_slot(key, a.mem_mask);
  for (int k = 0; k < kMemProbes; ++k) {
    const unsigned long long v = atomicCAS(&a.mem[h], kMemEmpty, key);
    if (v == kMemEmpty || v == key) return;
    h = (h + 1) & a.mem_mask;
  }
  atomicOr(a.status, DEM_DEV_FRONTIER_OVERFLOW);
}

// Exclusive prefix sums of v[0..n) in place, total to v[n]; one block of
// kScanThreads threads, each summing a contiguous slice first.
__device__ void block_scan_u64(unsigned long long* v, uint32_t n) {
  __shared__ unsigned long long wsum[kScanThreads / kWave];
  const uint32_t per = (n + blockDim.x - 1) / blockDim.x;
  const uint32_t lo = min(threadIdx.x * per, n), hi = min(lo + per, n);
  unsigned long long s = 0;
  for (uint32_t k = lo; k < hi; ++k) s += v[k];
  const int lane = lane_id(), wid = threadIdx.x / kWave;
  unsigned long long x = s;
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    unsigned long long y = __shfl_up(x, o);
    if (lane >= o) x += y;
  }
  if (lane == kWave - 1) wsum[wid] = x;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long acc = 0;
    for (int w = 0; w < (int)(blockDim.x / kWave); ++w) {
      unsigned long long t = wsum[w];
      wsum[w] = acc;
      acc += t;
    }
    v[n] = acc;
  }
  __syncthreads();
  unsigned long long run = x - s + wsum[wid];
  for (uint32_t k = lo; k < hi; ++k) {
    unsigned long long t = v[k];
    v[k] = run;
    run += t;
  }
}

// Contiguous leaf range of block b (a multiple of blockDim), so that the
// output keeps the depth-first order.
__device__ __forceinline__ void fr_range(uint32_t n, uint32_t& lo, uint32_t& hi) {
  const uint32_t G = gridDim.x, B = blockDim.x;
  const uint32_t per = ((n + G - 1) / G + B - 1) / B * B;
  lo = min((uint64_t)blockIdx.x * per, (uint64_t)n);
  hi = min((uint64_t)lo + per, (uint64_t)n);
}

template <typename T, int N, bool EXACT>
__global__ void __launch_bounds__(kFrBlock) k_fr_eval(const SoupRec<T>* __restrict__ soup, FrontierArgs a) {
  __shared__ LdsQueue<int2, kStageNear> qn;
  __shared__ uint32_t hist[DEM_MAX_LEVELS];
  const uint32_t n = fr_count(a);
  const int4* __restrict__ lin = a.state[0] ? a.buf1 : a.buf0;
  if (threadIdx.x == 0) qn.n = 0;
  if (threadIdx.x < DEM_MAX_LEVELS) hist[threadIdx.x] = 0;
  if (blockIdx.x == 0 && threadIdx.x == 0) a.state[2] = n;
  __syncthreads();
  uint32_t my_unf = 0, my_near = 0;
  unsigned long long my_out = 0;  // leaves this thread's leaves become if no group narrows
  uint32_t lo, hi;
  fr_range(n, lo, hi);
  for (uint32_t base = lo; base < hi; base += blockDim.x) {
    const uint32_t i = base + threadIdx.x;
    bool near = false;
    int dep = -1;  // the leaf's pair depth, for the per-depth evaluation counts
    const int4 lf = i < hi ? lin[i] : make_int4(0, 0, 0, 0);
    const bool valid = (uint32_t)lf.x < (uint32_t)a.n_tris && (uint32_t)lf.y < (uint32_t)a.n_tris;
    if (i < hi && !valid) {
      atomicOr(a.status, DEM_DEV_BAD_TREE);  // not a leaf this library wrote: the sets stay as they are
      a.meta[i] = kOutKeep;
      a.cm[i] = 0;
    }
    if (i < hi && valid) {
      int cbi, cci, pi_, cbj, ccj, pj_;
      Tri<T> A = load_tri(soup, lf.x, cbi, cci, pi_);
      Tri<T> B = load_tri(soup, lf.y, cbj, ccj, pj_);
      V3<T> D0 = A.v0 - B.v0;
      const T delta = A.eps + B.eps;
      bool keep;
      if constexpr (EXACT) {
        Closest<T> c;
        exact_tri_tri(V3<T>{0, 0, 0}, A.e1, A.e2, -D0, B.e1, B.e2, c);
        keep = !(sq_(c.d2) > delta);
      } else {
        const T L = iterate_bound<T, N>(A, B, D0, a.ip);
        keep = !(L > delta + bound_slack(A, B, D0, delta));
      }
      const uint32_t info = (uint32_t)lf.w, flags = (uint32_t)lf.z;
      const uint32_t D = fr_depth(info), g = fr_gidx(info), gn = fr_gsize(info);
      // first leaf of a group that may narrow (not vetoed by the memory set)
      const uint32_t head = (D >= 1 && g == 0 && gn >= 1 && !((flags >> D) & 1u)) ? gn : 0u;
      uint32_t out, nn;
      if (!keep) {
        out = kOutPrune; nn = head;
      } else if (cci == 0 && ccj == 0) {
        out = kOutNear; nn = head;  // settled by k_near
      } else {
        out = kOutUnfold; nn = (uint32_t)(cci ? cci : 1) * (uint32_t)(ccj ? ccj : 1);
      }
      a.meta[i] = out | (g << 8) | (nn << 16);
      a.cm[i] = 0;
      my_out += out == kOutUnfold ? nn : 1u;
      near = out == kOutNear;
      my_unf += out == kOutUnfold;
      my_near += near;
      if (D < (uint32_t)DEM_MAX_LEVELS) dep = (int)D;
    }
    if (a.stats) {
      // one LDS atomic per depth present in the wave (most lanes share one)
      unsigned long long pending = __ballot(dep >= 0);
      while (pending) {
        const int leader = __ffsll((long long)pending) - 1;
        const int d0 = __shfl(dep, leader);
        const unsigned long long same = __ballot(dep == d0) & pending;
        if (lane_id() == leader) atomicAdd(&hist[d0], (uint32_t)__popcll(same));
        pending &= ~same;
      }
    }
    lds_append(near, make_int2((int)i, 0), qn.buf, &qn.n);
    __syncthreads();
    if (qn.n + blockDim.x > (uint32_t)kStageNear)
      lds_flush(qn, a.near_tail, a.near_, a.ncap, a.status, DEM_DEV_NEAR_OVERFLOW);
  }
  __syncthreads();
  lds_flush(qn, a.near_tail, a.near_, a.ncap, a.status, DEM_DEV_NEAR_OVERFLOW);
  __shared__ unsigned long long osum[kFrBlock / kWave], nsum[kFrBlock / kWave];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    my_unf += __shfl_xor(my_unf, o);
    my_near += __shfl_xor(my_near, o);
    my_out += __shfl_xor(my_out, o);
  }
  if (lane_id() == 0) {
    osum[threadIdx.x / kWave] = my_out;
    nsum[threadIdx.x / kWave] = my_near;
    if (my_unf) atomicAdd(&a.ctr->fr_unfold, my_unf);  // (rare: the leaves that widen)
  }
  __syncthreads();
  // counts into this block's partial (k_fold_stats adds them up): one atomic
  // per wave on one address serialised across the whole grid
  StatPart* sp = a.spart ? &a.spart[blockIdx.x % kStatPart] : nullptr;
  if (threadIdx.x == 0) {
    unsigned long long t = 0, nr = 0;
    for (int w = 0; w < (int)(blockDim.x / kWave); ++w) {
      t += osum[w];
      nr += nsum[w];
    }
    a.part[blockIdx.x] = t;  // output leaves of this block's range, before narrowing
    if (a.stats && nr) atomicAdd(sp ? &sp->near : &a.stats->near, nr);
  }
  if (a.stats && threadIdx.x < DEM_MAX_LEVELS && hist[threadIdx.x])
    atomicAdd(sp ? &sp->evals[threadIdx.x] : &a.stats->evals[threadIdx.x], (unsigned long long)hist[threadIdx.x]);
  if (a.stats && blockIdx.x == 0 && threadIdx.x == 0) atomicAdd(&a.stats->frontier_leaves, (unsigned long long)n);
}

// Narrowing: a group's first leaf checks its n - 1 followers.  In depth-first
// order a member that is not a leaf is followed by its own first descendant
// leaf, whose group index is 0, so the check fails exactly when some member
// is not a leaf or not "no contact".  A narrowed group leaves one leaf
// instead of n: the output counts of the blocks holding its other members
// drop by one each (block ranges as in fr_range).
__global__ void __launch_bounds__(kFrBlock) k_fr_group(FrontierArgs a) {
  const uint32_t n = fr_count(a);
  const uint32_t G = gridDim.x, B = blockDim.x;
  const uint32_t per = ((n + G - 1) / G + B - 1) / B * B;
  const int lane = lane_id();
  uint32_t my = 0;
  // every wave takes 64 consecutive leaves per round (bounds are wave-uniform)
  for (uint32_t base = blockIdx.x * blockDim.x; base < n; base += gridDim.x * blockDim.x) {
    const uint32_t i = base + threadIdx.x;
    const uint32_t m = i < n ? a.meta[i] : 0xFFu;
    uint32_t prev = __shfl_up(m, 1);
    if (lane == 0) prev = (i >= 1 && i - 1 < n) ? a.meta[i - 1] : 0xFFu;
    const bool pr = (m & 255u) == kOutPrune;
    const uint32_t g = (m >> 8) & 255u;
    // link: "no contact", and the follower of the previous leaf in its group
    const bool link = pr && g >= 1 && (prev & 255u) == kOutPrune && ((prev >> 8) & 255u) == g - 1;
    const unsigned long long lm = __ballot(link);
    const uint32_t gn = m >> 16;
    if (!(i < n && pr && gn > 0 && g == 0 && (uint64_t)i + gn <= n)) continue;
    // members 1..gn-1 must all link up: lanes lane+1.. of this wave, then
    // loads for the part past the wave
    bool all;
    if ((uint32_t)lane + gn <= 64u) {
      const unsigned long long need = gn >= 2 ? ((1ull << (gn - 1)) - 1ull) << (lane + 1) : 0ull;
      all = (lm & need) == need;
    } else {
      const unsigned long long need = lane < 63 ? (~0ull << (lane + 1)) : 0ull;
      all = (lm & need) == need;
      for (uint32_t j = 64u - (uint32_t)lane; j < gn && all; ++j) {
        const uint32_t mj = a.meta[i + j];
        all = (mj & 255u) == kOutPrune && ((mj >> 8) & 255u) == j;
      }
    }
    if (!all) continue;
    a.cm[i] = 2;
    for (uint32_t j = 1; j < gn; ++j) {
      a.cm[i + j] = 1;
      atomicAdd(&a.part[(i + j) / per], ~0ull);  // -1
    }
    ++my;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) my += __shfl_xor(my, o);
  if (lane_id() == 0 && my) atomicAdd(&a.ctr->fr_collapse, my);
}

__device__ __forceinline__ bool fr_skip(const FrontierArgs& a) {
  constexpr uint32_t bad = DEM_DEV_NEAR_OVERFLOW | DEM_DEV_CONTACT_OVERFLOW | DEM_DEV_NONFINITE |
                           DEM_DEV_BAD_TREE | DEM_DEV_FRONTIER_OVERFLOW;
  return (a.ctr->fr_unfold == 0 && a.ctr->fr_collapse == 0) || (*a.status & bad) || a.ctr->fr_skip;
}

__device__ __forceinline__ uint32_t fr_out_count(uint32_t m, uint8_t c) {
  if (c == 2) return 1;
  if (c == 1) return 0;
  return (m & 255u) == kOutUnfold ? (m >> 16) : 1u;
}

__global__ void __launch_bounds__(kScanThreads) k_fr_scan(FrontierArgs a, uint32_t n_blocks) {
  if (fr_skip(a)) return;
  block_scan_u64(a.part, n_blocks);
  if (threadIdx.x == 0) {
    const unsigned long long total = a.part[n_blocks];
    a.state[2] = (uint32_t)min(total, 0xFFFFFFFFull);
    if (total > (unsigned long long)a.cap) {
      atomicOr(a.status, DEM_DEV_FRONTIER_OVERFLOW);
      a.ctr->fr_skip = 1;
    }
  }
}

__global__ void __launch_bounds__(kFrBlock) k_fr_emit(FrontierArgs a) {
  __shared__ int4 lf_s[kFrBlock];
  __shared__ uint32_t m_s[kFrBlock];
  __shared__ uint8_t c_s[kFrBlock];
  __shared__ int offs[kFrBlock + 1];
  __shared__ int wsum[kFrBlock / kWave];
  __shared__ int skip;
  // one decision per block: the status word may gain a memory-set overflow
  // bit from other blocks while this kernel runs
  if (threadIdx.x == 0) skip = fr_skip(a);
  __syncthreads();
  if (skip) return;
  const uint32_t cur = a.state[0];
  const int4* __restrict__ lin = cur ? a.buf1 : a.buf0;
  int4* __restrict__ lout = cur ? a.buf0 : a.buf1;
  uint32_t lo, hi;
  fr_range(fr_count(a), lo, hi);
  unsigned long long obase = a.part[blockIdx.x];
  const int B = blockDim.x;
  for (uint32_t t0 = lo; t0 < hi; t0 += B) {
    const uint32_t i = t0 + threadIdx.x;
    int c = 0;
    if (i < hi) {
      lf_s[threadIdx.x] = lin[i];
      m_s[threadIdx.x] = a.meta[i];
      c_s[threadIdx.x] = a.cm[i];
      c = (int)fr_out_count(m_s[threadIdx.x], c_s[threadIdx.x]);
    }
    // a tile without widening or narrowing is copied as it is
    const bool plain = i >= hi || (c_s[threadIdx.x] == 0 && (m_s[threadIdx.x] & 255u) != kOutUnfold);
    if (__syncthreads_and(plain)) {
      if (i < hi) lout[obase + (i - t0)] = lf_s[threadIdx.x];
      obase += min((uint32_t)B, hi - t0);
      __syncthreads();
      continue;
    }
    block_scan(c, offs, wsum, B);
    const int total = offs[B];
    for (int e = threadIdx.x; e < total; e += B) {
      // owner: last k with offs[k] <= e (zero-count entries before it share offsets)
      int lo2 = 0, hi2 = B - 1;
      while (lo2 < hi2) {
        int mid = (lo2 + hi2 + 1) >> 1;
        if (offs[mid] <= e) lo2 = mid; else hi2 = mid - 1;
      }
      const int4 lf = lf_s[lo2];
      const uint32_t m = m_s[lo2];
      const uint32_t l = (uint32_t)(e - offs[lo2]);
      const uint32_t flags = (uint32_t)lf.z, info = (uint32_t)lf.w;
      const uint32_t D = fr_depth(info);
      int4 r = lf;
      if (c_s[lo2] == 2) {
        // narrowing: the group's parent pair, now in the memory set
        const int pa = (info >> 22) & 1u ? a.tri_parent[lf.x] : lf.x;
        const int pb = (info >> 23) & 1u ? a.tri_parent[lf.y] : lf.y;
        const uint32_t D1 = D - 1;
        uint32_t ninfo = 0;
        if (D1 > 0) {
          const uint32_t sa = a.tri_depth[pa] == D1, sb = a.tri_depth[pb] == D1;
          const int ppa = sa ? a.tri_parent[pa] : pa, ppb = sb ? a.tri_parent[pb] : pb;
          const uint32_t na = sa ? (uint32_t)a.ccnt[ppa] : 1u, nb = sb ? (uint32_t)a.ccnt[ppb] : 1u;
          const uint32_t ia = sa ? (uint32_t)(pa - a.cbeg[ppa]) : 0u, ib = sb ? (uint32_t)(pb - a.cbeg[ppb]) : 0u;
          ninfo = fr_info(ia * nb + ib, na * nb, D1, sa, sb);
        }
        mem_insert(a, mem_key(pa, pb));
        r = make_int4(pa, pb, (int)((flags & ((1u << D) - 1u)) | 1u), (int)ninfo);
      } else if ((m & 255u) == kOutUnfold) {
        // widening: child pair l, children of a non-fine side only
        const int na = a.ccnt[lf.x], nb = a.ccnt[lf.y];
        const uint32_t si = na > 0, sj = nb > 0;
        const uint32_t nbj = sj ? (uint32_t)nb : 1u;
        const uint32_t ia = l / nbj, ib = l - ia * nbj;
        const int ca = si ? a.cbeg[lf.x] + (int)ia : lf.x;
        const int cb = sj ? a.cbeg[lf.y] + (int)ib : lf.y;
        const uint32_t D1 = D + 1;
        const uint32_t nflags = (flags & ~1u) | ((flags & 1u) << D1) | (mem_contains(a, mem_key(ca, cb)) ? 1u : 0u);
        r = make_int4(ca, cb, (int)nflags, (int)fr_info(l, m >> 16, D1, si, sj));
      }
      lout[obase + (unsigned long long)e] = r;
    }
    obase += (unsigned long long)total;
    __syncthreads();
  }
}

__global__ void k_fr_finish(FrontierArgs a) {
  if (threadIdx.x != 0) return;
  if (a.stats) {
    a.stats->frontier_unfolded = a.ctr->fr_unfold;
    a.stats->frontier_collapsed = a.ctr->fr_collapse;
  }
  if (fr_skip(a)) return;
  a.state[0] ^= 1u;
  a.state[1] = a.state[2];
}

// Initial active sets: every root pair of every candidate pair.
__global__ void k_fr_init_count(const int32_t* __restrict__ pairs, int n_pairs, const int32_t* __restrict__ rcnt,
                                unsigned long long* pc) {
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < n_pairs; k += gridDim.x * blockDim.x)
    pc[k] = (unsigned long long)rcnt[pairs[k]] * (unsigned long long)rcnt[pairs[n_pairs + k]];
}

__global__ void __launch_bounds__(kScanThreads) k_fr_init_scan(unsigned long long* pc, int n_pairs, uint32_t* state,
                                                                int64_t cap, uint32_t* status) {
  block_scan_u64(pc, (uint32_t)n_pairs);
  if (threadIdx.x == 0) {
    const unsigned long long total = pc[n_pairs];
    state[0] = 0;
    state[2] = (uint32_t)min(total, 0xFFFFFFFFull);
    state[3] = 0;
    if (total > (unsigned long long)cap) {
      state[1] = 0;
      *status = DEM_DEV_FRONTIER_OVERFLOW;
    } else {
      state[1] = (uint32_t)total;
      *status = 0;
    }
  }
}

__global__ void k_fr_init_write(const int32_t* __restrict__ pairs, int n_pairs, const int32_t* __restrict__ rbeg,
                                const int32_t* __restrict__ rcnt, const unsigned long long* __restrict__ pc,
                                int64_t cap, int4* __restrict__ out) {
  if (pc[n_pairs] > (unsigned long long)cap) return;
  for (int k = blockIdx.x; k < n_pairs; k += gridDim.x) {
    const int pi = pairs[k], pj = pairs[n_pairs + k];
    const int bi = rbeg[pi], ni = rcnt[pi], bj = rbeg[pj], nj = rcnt[pj];
    for (int e = threadIdx.x; e < ni * nj; e += blockDim.x) {
      const int ii = e / nj, jj = e - ii * nj;
      out[pc[k] + (unsigned long long)e] = make_int4(bi + ii, bj + jj, 0, 0);
    }
  }
}

__global__ void k_fr_mem_clear(unsigned long long* mem, int64_t n) {
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x)
    mem[k] = kMemEmpty;
}

// ------------------------------------------------------------------ contact forces
// dem_contact_forces (Section 2: force of a contact point, merging of
// redundant points).  Cells are cubes of side r / sqrt(3) (r = the merge
// radius of the particle pair), shrunk by 1e-5, so two points of one cell are
// closer than r and a cell's points belong to one group without any test.
//   k_cf_clear   empty the cell table (hash of (particle pair, cell) keys)
//   k_cf_insert  every contact's key into the table; points per slot
//   k_cf_range   every occupied slot a compact cell id and a contiguous range
//                of the point order (blocks take contiguous slot chunks and
//                reserve their ids and ranges with one atomic each)
//   k_cf_place   every contact into its cell's range
//   k_cf_cells   per cell (one wave, lanes over the points): smallest
//                contact index m, the cell record (coordinates, bounding box,
//                radius, pair), its point and normal sums (FP64) kept at m;
//                the union-find runs over the m's (the cells start as stars);
//                a 64-bit key collision is reported
//   k_cf_link    per (cell, neighbouring cell) with offsets up to 2 in one
//                half-space (each cell pair once): if the boxes come closer
//                than r and some pair of their points is closer than r, the
//                two cells join (union-find, links from the larger root to
//                the smaller: a group's root is its smallest contact index);
//                adjacent offsets first, then k_cf_compress, then the others
//   k_cf_sum     per cell: its group root, and its sums added at the root
//   k_cf_emit    one merged contact per root: mean point and normal, the
//                force, per-particle force and torque
//   k_cf_group   merged index of every input contact (optional output)
constexpr unsigned long long kCellEmpty = ~0ull;
constexpr int kCellProbes = 64;
constexpr int kNbr = 62;                    // neighbouring cells of one half-space
constexpr uint32_t kLinkBudget = 1u << 16;  // parent reads per thread in one kernel
constexpr double kCellShrink = 0.57735026918962576 * (1.0 - 1e-5);  // cell side / r

// Per-cell record (k_cf_cells writes it, k_cf_link reads it): cell
// coordinates, bounding box of the points, merge radius, smallest contact and
// particle pair.  64 B in FP32, 96 B in FP64.
template <typename T>
struct alignas(16) CellRec {
  long long cx, cy, cz;
  T lo[3], hi[3];
  T r;
  int32_t cmin, pi, pj;
};

template <typename T>
struct ForceArgs {
  const int32_t* pi;
  const int32_t* pj;
  const int32_t* ti;
  const int32_t* tj;
  const T* x;          // [3][ccap]
  const T* n;
  int64_t ccap;
  const uint32_t* ccount;
  const T* teps;
  int n_tris;
  T scale;
  // cell table (tmask + 1 slots)
  unsigned long long* keys;
  uint32_t* scnt;      // points per slot
  int32_t* sid;        // compact cell id of an occupied slot
  uint64_t tmask;
  uint32_t* n_cells;   // [2]: cells, points placed
  // cells (compact ids, up to ccap)
  uint32_t* coff;      // first position of the cell's range
  uint32_t* ccnt;
  uint32_t* cfill;
  int32_t* cmin;       // smallest contact index of the cell
  CellRec<T>* crec;    // [ccap]
  // per contact
  int32_t* pcell;      // cell id of the contact (-1: none)
  int32_t* order;      // contacts ordered by cell
  T* pts;              // [ccap][8] in cell order: point x, y, z, pi, normal x, y, z, pj
  int32_t* parent;
  int32_t* root;       // group root of every cell (by cell id)
  int32_t* mslot;
  double* acc;         // [7][ccap]: point sums, normal sums, members (at group roots)
  // force law
  const T* mass;
  const T* centre;     // [3][n_particles]
  int n_particles;
  T k_s;
  // outputs
  int32_t* opi;
  int32_t* opj;
  T* ox;
  T* on;
  T* of;
  int32_t* omem;
  uint32_t* ocount;
  int64_t ocap;
  int32_t* group;
  T* force;
  T* torque;
  uint32_t* status;
};

// One half of a cell-ordered point record (16 B in FP32, 32 B in FP64).
template <typename T>
struct alignas(4 * sizeof(T)) Q4 {
  T x, y, z, w;
};

// The records' fourth words carry the contact's particles (pi in the point
// half, pj in the normal half), as integer bits.
__device__ __forceinline__ float int_bits(int v, float) { return __int_as_float(v); }
__device__ __forceinline__ double int_bits(int v, double) { return __longlong_as_double((long long)v); }
__device__ __forceinline__ int bits_int(float v) { return __float_as_int(v); }
__device__ __forceinline__ int bits_int(double v) { return (int)__double_as_longlong(v); }

template <typename T>
__device__ __forceinline__ Q4<T> cf_pt(const ForceArgs<T>& a, size_t pos) {
  return reinterpret_cast<const Q4<T>*>(a.pts)[2 * pos];
}

template <typename T>
__device__ __forceinline__ Q4<T> cf_nr(const ForceArgs<T>& a, size_t pos) {
  return reinterpret_cast<const Q4<T>*>(a.pts)[2 * pos + 1];
}

__device__ __forceinline__ unsigned long long mix64(unsigned long long z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__device__ __forceinline__ unsigned long long cell_key(int pi, int pj, long long cx, long long cy, long long cz) {
  unsigned long long h = mix64(((unsigned long long)(uint32_t)pi << 32) | (uint32_t)pj);
  h = mix64(h ^ (unsigned long long)cx);
  h = mix64(h ^ (unsigned long long)cy);
  h = mix64(h ^ (unsigned long long)cz);
  return h == kCellEmpty ? h ^ 1ull : h;
}

template <typename T>
__device__ __forceinline__ uint32_t cf_count(const ForceArgs<T>& a) {
  return (uint32_t)min((uint64_t)*a.ccount, (uint64_t)a.ccap);
}

// Whether contact c names triangles and particles this scene has (else it is
// skipped and flagged).
template <typename T>
__device__ __forceinline__ bool cf_valid(const ForceArgs<T>& a, uint32_t c) {
  return (uint32_t)a.ti[c] < (uint32_t)a.n_tris && (uint32_t)a.tj[c] < (uint32_t)a.n_tris &&
         (uint32_t)a.pi[c] < (uint32_t)a.n_particles && (uint32_t)a.pj[c] < (uint32_t)a.n_particles;
}

// Merge radius of the contact's particle pair: scale * (eps_i + eps_j) / 2.
template <typename T>
__device__ __forceinline__ T cf_radius(const ForceArgs<T>& a, uint32_t c) {
  return a.scale * T(0.5) * (a.teps[a.ti[c]] + a.teps[a.tj[c]]);
}

template <typename T>
__device__ __forceinline__ void cf_cell(const ForceArgs<T>& a, uint32_t c, T r, long long& cx, long long& cy,
                                        long long& cz) {
  const T inv = T(1) / (r * T(kCellShrink));
  cx = (long long)floor(a.x[c] * inv);
  cy = (long long)floor(a.x[a.ccap + c] * inv);
  cz = (long long)floor(a.x[2 * a.ccap + c] * inv);
}

// Cell id of a key, -1 if absent.  A probe loads the slot's key and cell id
// together (the id is used only if the key matches).
template <typename T>
__device__ __forceinline__ int cf_find_id(const ForceArgs<T>& a, unsigned long long key) {
  uint64_t slot = mix64(key) & a.tmask;
  for (int k = 0; k < kCellProbes; ++k) {
    const unsigned long long kk = a.keys[slot];
    const int id = a.sid[slot];
    if (kk == key) return id;
    if (kk == kCellEmpty) return -1;
    slot = (slot + 1) & a.tmask;
  }
  return -1;
}

// Root of x (device-coherent reads: parents change under other lanes'
// links); path halving stores ancestors only.  Parents have smaller indices
// than their children, so there are no cycles.  -1 when the budget runs out.
__device__ int uf_root(int32_t* parent, int x, uint32_t& budget) {
  while (budget) {
    --budget;
    const int p = __hip_atomic_load(parent + x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (p == x) return x;
    const int g = __hip_atomic_load(parent + p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (g != p) __hip_atomic_store(parent + x, g, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    x = g;
  }
  return -1;
}

// Root estimate from plain (possibly stale) reads: equal estimates for two
// points prove they are already in one group (groups only ever join).
__device__ __forceinline__ int uf_root_plain(const int32_t* parent, int x) {
  for (int k = 0; k < 64; ++k) {
    const int p = parent[x];
    if (p == x) return x;
    x = p;
  }
  return -1;
}

__device__ void uf_union(int32_t* parent, int a, int b, uint32_t& budget, uint32_t* status) {
  while (budget) {
    a = uf_root(parent, a, budget);
    b = uf_root(parent, b, budget);
    if (a < 0 || b < 0) break;
    if (a == b) return;
    const int hi = max(a, b), lo = min(a, b);
    if (atomicCAS(parent + hi, hi, lo) == hi) return;
  }
  atomicOr(status, DEM_DEV_QUEUE_OVERFLOW);
}

template <typename T>
__global__ void k_cf_clear(ForceArgs<T> a, uint64_t n) {
  for (uint64_t k = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; k < n; k += (uint64_t)gridDim.x * blockDim.x) {
    a.keys[k] = kCellEmpty;
    a.scnt[k] = 0;
  }
  if (blockIdx.x == 0 && threadIdx.x < 2) a.n_cells[threadIdx.x] = 0;
}

// Contacts next to each other in the list mostly share a cell: a run of
// lanes with one key is served by its first lane (one probe sequence, one
// count update for the run); the runs' leaders work in parallel.
template <typename T>
__global__ void __launch_bounds__(256) k_cf_insert(ForceArgs<T> a) {
  const uint32_t cnt = cf_count(a);
  const int lane = lane_id();
  for (uint32_t base = blockIdx.x * blockDim.x; base < cnt; base += gridDim.x * blockDim.x) {
    const uint32_t c = base + threadIdx.x;
    bool has = false;
    unsigned long long key = 0;
    if (c < cnt) {
      a.pcell[c] = -1;
      if (!cf_valid(a, c)) {
        atomicOr(a.status, DEM_DEV_BAD_TREE);
      } else if (a.scale > T(0)) {
        const T r = cf_radius(a, c);
        if (r > T(0)) {
          long long cx, cy, cz;
          cf_cell(a, c, r, cx, cy, cz);
          key = cell_key(a.pi[c], a.pj[c], cx, cy, cz);
          has = true;
        }
      }
    }
    const unsigned long long prev_key = __shfl_up(key, 1);
    const bool prev_has = __shfl_up((int)has, 1) != 0;
    const bool lead = has && (lane == 0 || !prev_has || prev_key != key);
    const unsigned long long leaders = __ballot(lead), members = __ballot(has);
    // a leader's run: it and the following lanes up to the next leader or gap
    const unsigned long long after = lane == 63 ? 0ull : (~0ull << (lane + 1));
    const unsigned long long stops = (leaders | ~members) & after;
    const int end = stops ? __ffsll((long long)stops) - 1 : 64;
    int slot = -1;
    if (lead) {
      uint64_t sl = mix64(key) & a.tmask;
      for (int k = 0; k < kCellProbes; ++k) {
        const unsigned long long old = atomicCAS(a.keys + sl, kCellEmpty, key);
        if (old == kCellEmpty || old == key) {
          slot = (int)sl;
          break;
        }
        sl = (sl + 1) & a.tmask;
      }
      if (slot < 0) atomicOr(a.status, DEM_DEV_QUEUE_OVERFLOW);
      else atomicAdd(a.scnt + slot, (uint32_t)(end - lane));
    }
    // every member takes its run leader's slot
    const unsigned long long upto = lane == 63 ? ~0ull : ((2ull << lane) - 1ull);
    const int my_lead = 63 - __clzll((long long)(leaders & upto));
    slot = __shfl(slot, has ? my_lead : lane);
    if (has && slot >= 0) a.pcell[c] = slot;  // a slot for now; k_cf_place turns it into a cell id
  }
}

// Block sum of v over the whole block (every thread gets it).
__device__ __forceinline__ unsigned long long block_sum_u64(unsigned long long v, unsigned long long* red) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  if (lane_id() == 0) red[threadIdx.x / kWave] = v;
  __syncthreads();
  unsigned long long t = 0;
  for (int w = 0; w < (int)(blockDim.x / kWave); ++w) t += red[w];
  __syncthreads();
  return t;
}

template <typename T>
__global__ void __launch_bounds__(256) k_cf_range(ForceArgs<T> a, uint64_t n) {
  __shared__ unsigned long long red[256 / kWave];
  __shared__ int woff[256 / kWave][2];
  __shared__ uint32_t base_c, base_p;
  const uint64_t per = (n + gridDim.x - 1) / gridDim.x;
  const uint64_t lo = min(blockIdx.x * per, n), hi = min(lo + per, n);
  // pass 1: cells and points of this block's chunk
  unsigned long long mc = 0, mp = 0;
  for (uint64_t s = lo + threadIdx.x; s < hi; s += blockDim.x) {
    const uint32_t m = a.scnt[s];
    mc += m ? 1u : 0u;
    mp += m;
  }
  const unsigned long long tc = block_sum_u64(mc, red);
  const unsigned long long tp = block_sum_u64(mp, red);
  if (threadIdx.x == 0) {
    base_c = tc ? atomicAdd(a.n_cells, (uint32_t)tc) : 0u;
    base_p = tp ? atomicAdd(a.n_cells + 1, (uint32_t)tp) : 0u;
  }
  __syncthreads();
  // pass 2: hand out ids and ranges in slot order, a block-wide round at a time
  uint32_t run_c = base_c, run_p = base_p;
  for (uint64_t t0 = lo; t0 < hi; t0 += blockDim.x) {
    const uint64_t s = t0 + threadIdx.x;
    const uint32_t m = s < hi ? a.scnt[s] : 0u;
    uint32_t vc = m ? 1u : 0u, vp = m;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
      const uint32_t yc = __shfl_up(vc, o), yp = __shfl_up(vp, o);
      if (lane_id() >= o) { vc += yc; vp += yp; }
    }
    const int w = threadIdx.x / kWave;
    if (lane_id() == kWave - 1) { woff[w][0] = (int)vc; woff[w][1] = (int)vp; }
    __syncthreads();
    uint32_t pc = 0, pp = 0, tcr = 0, tpr = 0;
    for (int k = 0; k < (int)(blockDim.x / kWave); ++k) {
      if (k < w) { pc += (uint32_t)woff[k][0]; pp += (uint32_t)woff[k][1]; }
      tcr += (uint32_t)woff[k][0];
      tpr += (uint32_t)woff[k][1];
    }
    if (m) {
      const uint32_t id = run_c + pc + vc - 1u;
      a.sid[s] = (int32_t)id;
      a.coff[id] = run_p + pp + vp - m;
      a.ccnt[id] = m;
      a.cfill[id] = 0;
    }
    run_c += tcr;
    run_p += tpr;
    __syncthreads();
  }
}

// Positions within a cell's range: one count update per run of lanes with
// one cell (its first lane's, all runs in parallel), lanes ranked in the run.
template <typename T>
__global__ void __launch_bounds__(256) k_cf_place(ForceArgs<T> a) {
  const uint32_t cnt = cf_count(a);
  const int lane = lane_id();
  for (uint32_t base = blockIdx.x * blockDim.x; base < cnt; base += gridDim.x * blockDim.x) {
    const uint32_t c = base + threadIdx.x;
    int id = -1;
    if (c < cnt) {
      const int slot = a.pcell[c];
      if (slot >= 0) id = a.sid[slot];
    }
    const bool act = id >= 0;
    const int prev_id = __shfl_up(id, 1);
    const bool lead = act && (lane == 0 || prev_id != id);
    const unsigned long long leaders = __ballot(lead), members = __ballot(act);
    const unsigned long long after = lane == 63 ? 0ull : (~0ull << (lane + 1));
    const unsigned long long stops = (leaders | ~members) & after;
    const int end = stops ? __ffsll((long long)stops) - 1 : 64;
    uint32_t b = 0;
    if (lead) b = a.coff[id] + atomicAdd(a.cfill + id, (uint32_t)(end - lane));
    const unsigned long long upto = lane == 63 ? ~0ull : ((2ull << lane) - 1ull);
    const int my_lead = 63 - __clzll((long long)(leaders & upto));
    b = __shfl(b, act ? my_lead : lane);
    if (!act) continue;
    const uint32_t pos = b + (uint32_t)(lane - my_lead);
    a.pcell[c] = id;
    a.order[pos] = (int32_t)c;
    const size_t C = (size_t)a.ccap;
    Q4<T>* q = reinterpret_cast<Q4<T>*>(a.pts) + 2 * (size_t)pos;
    q[0] = Q4<T>{a.x[c], a.x[C + c], a.x[2 * C + c], int_bits(a.pi[c], T(0))};
    q[1] = Q4<T>{a.n[c], a.n[C + c], a.n[2 * C + c], int_bits(a.pj[c], T(0))};
  }
}

// Reductions over the 16 lanes of a DPP row, every lane getting the result:
// lanes i ^ 1 and i ^ 2 (quad permutations), then i and 7 - i within each
// half row, then i and 15 - i within the row.  All 16 lanes must be active.
template <int CTRL>
__device__ __forceinline__ int dpp_row(int v) {
  return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, false);
}
template <int CTRL>
__device__ __forceinline__ float dpp_row(float v) {
  return __int_as_float(dpp_row<CTRL>(__float_as_int(v)));
}
template <int CTRL>
__device__ __forceinline__ double dpp_row(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = dpp_row<CTRL>((int)b), hi = dpp_row<CTRL>((int)(b >> 32));
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned int)lo);
}
struct OpMin {
  template <typename V>
  __device__ V operator()(V x, V y) const { return min(x, y); }
};
struct OpMax {
  template <typename V>
  __device__ V operator()(V x, V y) const { return max(x, y); }
};
struct OpAdd {
  template <typename V>
  __device__ V operator()(V x, V y) const { return x + y; }
};
template <typename V, typename Op>
__device__ __forceinline__ V row_reduce(V v, Op op) {
  v = op(v, dpp_row<0xB1>(v));   // quad_perm [1, 0, 3, 2]
  v = op(v, dpp_row<0x4E>(v));   // quad_perm [2, 3, 0, 1]
  v = op(v, dpp_row<0x141>(v));  // row_half_mirror
  v = op(v, dpp_row<0x140>(v));  // row_mirror
  return v;
}

// One DPP row (16 lanes) per cell, lanes over its points.
constexpr uint32_t kCellLanes = 16;

template <typename T>
__global__ void __launch_bounds__(256) k_cf_cells(ForceArgs<T> a) {
  const uint32_t nc = a.n_cells[0];
  const uint32_t cnt = cf_count(a);
  const uint32_t sl = (uint32_t)lane_id() % kCellLanes;
  const uint32_t gpb = blockDim.x / kCellLanes, ng = gridDim.x * gpb;
  const size_t C = (size_t)a.ccap;
  for (uint32_t id = blockIdx.x * gpb + threadIdx.x / kCellLanes; id < nc; id += ng) {
    const uint32_t m = a.ccnt[id], o = a.coff[id];
    const int32_t* pts = a.order + o;
    int mn = INT_MAX;
    T lo[3] = {T(INFINITY), T(INFINITY), T(INFINITY)}, hi[3] = {-T(INFINITY), -T(INFINITY), -T(INFINITY)};
    double sm[7] = {0, 0, 0, 0, 0, 0, 0};  // the cell's point and normal sums, count
    for (uint32_t k = sl; k < m; k += kCellLanes) {
      mn = min(mn, pts[k]);
      const Q4<T> q = cf_pt(a, o + k), w = cf_nr(a, o + k);
      lo[0] = min(lo[0], q.x); lo[1] = min(lo[1], q.y); lo[2] = min(lo[2], q.z);
      hi[0] = max(hi[0], q.x); hi[1] = max(hi[1], q.y); hi[2] = max(hi[2], q.z);
      sm[0] += (double)q.x; sm[1] += (double)q.y; sm[2] += (double)q.z;
      sm[3] += (double)w.x; sm[4] += (double)w.y; sm[5] += (double)w.z;
      sm[6] += 1.0;
    }
    mn = row_reduce(mn, OpMin());
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      lo[d] = row_reduce(lo[d], OpMin());
      hi[d] = row_reduce(hi[d], OpMax());
    }
#pragma unroll
    for (int d = 0; d < 7; ++d) sm[d] = row_reduce(sm[d], OpAdd());
    if ((uint32_t)mn >= cnt) {  // never expected: keep the indices below valid
      if (sl == 0) atomicOr(a.status, DEM_DEV_QUEUE_OVERFLOW);
      mn = pts[0];
    }
    // one (pair, cell) per cell, else the 64-bit keys of two cells collided
    const T r = cf_radius(a, (uint32_t)mn);
    const T inv = T(1) / (r * T(kCellShrink));
    const int pi = a.pi[mn], pj = a.pj[mn];
    const long long cx = (long long)floor(a.x[mn] * inv), cy = (long long)floor(a.x[C + mn] * inv),
                    cz = (long long)floor(a.x[2 * C + mn] * inv);
    int same = 1;
    for (uint32_t k = sl; k < m; k += kCellLanes) {
      const Q4<T> q = cf_pt(a, o + k), w = cf_nr(a, o + k);
      same &= bits_int(q.w) == pi && bits_int(w.w) == pj && (long long)floor(q.x * inv) == cx &&
              (long long)floor(q.y * inv) == cy && (long long)floor(q.z * inv) == cz;
    }
    same = row_reduce(same, OpMin());
    if (sl == 0) {
      if (!same) atomicOr(a.status, DEM_DEV_QUEUE_OVERFLOW);
      a.cmin[id] = mn;
      a.parent[mn] = mn;  // union-find runs over the cells' smallest contacts only
    }
    // the cell's sums at its smallest contact; k_cf_sum moves them to the group root
    if (sl < 7) {
      double v = sm[0];
#pragma unroll
      for (int d = 1; d < 7; ++d) v = sl == (uint32_t)d ? sm[d] : v;
      a.acc[(size_t)sl * C + mn] = v;
    }
    if (sl == 7) {
      CellRec<T> cr;
      cr.cx = cx; cr.cy = cy; cr.cz = cz;
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        cr.lo[d] = lo[d];
        cr.hi[d] = hi[d];
      }
      cr.r = r;
      cr.cmin = mn; cr.pi = pi; cr.pj = pj;
      a.crec[id] = cr;
    }
  }
}

// Neighbour offsets (dx, dy, dz) of one half-space ((dz, dy, dx)
// lexicographically after zero), |d| <= 2 per axis: the 13 adjacent ones
// (largest |d| = 1) first, then the 49 others.
constexpr int kNbrAdjacent = 13;
constexpr int kLinkLanes = 16;                 // lanes per neighbour in k_cf_link's point tests
constexpr int kLinkGroups = kWave / kLinkLanes;
static_assert(kNbrAdjacent <= 64 && kNbr - kNbrAdjacent <= 64, "one lane per offset in k_cf_link");
__constant__ signed char kCfOff[kNbr][3] = {
    {1, 0, 0}, {-1, 1, 0}, {0, 1, 0}, {1, 1, 0}, {-1, -1, 1}, {0, -1, 1}, {1, -1, 1}, {-1, 0, 1},
    {0, 0, 1}, {1, 0, 1}, {-1, 1, 1}, {0, 1, 1}, {1, 1, 1}, {2, 0, 0}, {-2, 1, 0}, {2, 1, 0},
    {-2, 2, 0}, {-1, 2, 0}, {0, 2, 0}, {1, 2, 0}, {2, 2, 0}, {-2, -2, 1}, {-1, -2, 1}, {0, -2, 1},
    {1, -2, 1}, {2, -2, 1}, {-2, -1, 1}, {2, -1, 1}, {-2, 0, 1}, {2, 0, 1}, {-2, 1, 1}, {2, 1, 1},
    {-2, 2, 1}, {-1, 2, 1}, {0, 2, 1}, {1, 2, 1}, {2, 2, 1}, {-2, -2, 2}, {-1, -2, 2}, {0, -2, 2},
    {1, -2, 2}, {2, -2, 2}, {-2, -1, 2}, {-1, -1, 2}, {0, -1, 2}, {1, -1, 2}, {2, -1, 2}, {-2, 0, 2},
    {-1, 0, 2}, {0, 0, 2}, {1, 0, 2}, {2, 0, 2}, {-2, 1, 2}, {-1, 1, 2}, {0, 1, 2}, {1, 1, 2},
    {2, 1, 2}, {-2, 2, 2}, {-1, 2, 2}, {0, 2, 2}, {1, 2, 2}, {2, 2, 2}};

// One wave per cell A.  Lane l takes neighbour offset k0 + l (k1 - k0 <= 64)
// for the cheap tests: the neighbouring cell exists, its box comes closer
// than r to A's box, and the two are not yet one group.  The neighbours that
// pass are then taken kLinkGroups at a time, kLinkLanes lanes each: the
// lanes hold A's points (those within r of the neighbour's box) and scan the
// neighbour's points until one of them finds a point closer than r; one is
// enough to join the cells.
template <typename T>
__global__ void __launch_bounds__(256) k_cf_link(ForceArgs<T> a, int k0, int k1) {
  const uint32_t nc = a.n_cells[0];
  const int lane = lane_id();
  const uint32_t wpb = blockDim.x / kWave;
  const uint32_t nw = gridDim.x * wpb;
  for (uint32_t A = blockIdx.x * wpb + threadIdx.x / kWave; A < nc; A += nw) {
    const CellRec<T> ca = a.crec[A];
    const int ma = ca.cmin;
    const T r2 = ca.r * ca.r;
    const int pi = ca.pi, pj = ca.pj;
    const int k = k0 + lane;
    int B = -1, mb = -1;
    if (k < k1) {
      const int b = cf_find_id(a, cell_key(pi, pj, ca.cx + kCfOff[k][0], ca.cy + kCfOff[k][1], ca.cz + kCfOff[k][2]));
      if (b >= 0) {
        const CellRec<T> cb = a.crec[b];
        const int m = cb.cmin;
        if (cb.pi == pi && cb.pj == pj) {  // else a colliding key (reported by k_cf_cells)
          T gap2 = T(0);
#pragma unroll
          for (int d = 0; d < 3; ++d) {
            const T g = max(max(cb.lo[d] - ca.hi[d], ca.lo[d] - cb.hi[d]), T(0));
            gap2 += g * g;
          }
          if (gap2 < r2) {
            const int ra = uf_root_plain(a.parent, ma), rb = uf_root_plain(a.parent, m);
            if (!(ra >= 0 && ra == rb)) {
              B = b;
              mb = m;
            }
          }
        }
      }
    }
    // the remaining neighbours, kLinkGroups at a time: group g (kLinkLanes
    // lanes) takes the g-th lowest of them
    unsigned long long todo = __ballot(B >= 0);
    const size_t oa = a.coff[A];
    const uint32_t na = a.ccnt[A];
    const int grp = lane / kLinkLanes, gl = lane % kLinkLanes;
    const unsigned long long gmask = (kLinkLanes == 64 ? ~0ull : ((1ull << kLinkLanes) - 1ull)) << (grp * kLinkLanes);
    while (todo) {
      unsigned long long t = todo;
      for (int q = 0; q < grp && t; ++q) t &= t - 1;
      const int src = t ? __ffsll((long long)t) - 1 : 0;
#pragma unroll
      for (int q = 0; q < kLinkGroups; ++q) todo &= todo ? todo - 1 : 0ull;
      const int Bg = __shfl(B, src), mbg = __shfl(mb, src);
      bool live = t != 0ull;
      // an earlier neighbour may have joined them already
      if (live) {
        const int ra = uf_root_plain(a.parent, ma), rb = uf_root_plain(a.parent, mbg);
        live = !(ra >= 0 && ra == rb);
      }
      T bl[3] = {T(0), T(0), T(0)}, bh[3] = {T(0), T(0), T(0)};
      size_t ob = 0;
      uint32_t nb = 0;
      if (live) {
        const CellRec<T> cb = a.crec[Bg];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          bl[d] = cb.lo[d];
          bh[d] = cb.hi[d];
        }
        ob = a.coff[Bg];
        nb = a.ccnt[Bg];
      }
      bool close = false;
      // group-uniform loops: lanes gl, gl + kLinkLanes, ... over A's points
      for (uint32_t i0 = 0; live && i0 < na; i0 += kLinkLanes) {
        const uint32_t i = i0 + (uint32_t)gl;
        T xp = T(0), yp = T(0), zp = T(0);
        bool act = i < na;
        if (act) {
          const Q4<T> q = cf_pt(a, oa + i);
          xp = q.x;
          yp = q.y;
          zp = q.z;
          const T gx = max(max(bl[0] - xp, xp - bh[0]), T(0));
          const T gy = max(max(bl[1] - yp, yp - bh[1]), T(0));
          const T gz = max(max(bl[2] - zp, zp - bh[2]), T(0));
          act = gx * gx + gy * gy + gz * gz < r2;
        }
        if ((__ballot(act) & gmask) == 0ull) continue;
        for (uint32_t j = 0; j < nb; ++j) {
          const Q4<T> q = cf_pt(a, ob + j);
          const T ex = q.x - xp, ey = q.y - yp, ez = q.z - zp;
          close = close || (act && ex * ex + ey * ey + ez * ez < r2);
          if ((j & 7u) == 7u && (__ballot(close) & gmask) != 0ull) break;
        }
        if ((__ballot(close) & gmask) != 0ull) break;
      }
      const bool joined = (__ballot(close) & gmask) != 0ull;
      if (joined && gl == 0) {
        uint32_t budget = kLinkBudget;
        uf_union(a.parent, ma, mbg, budget, a.status);
      }
    }
  }
}


// Between the two linking launches: every cell's smallest contact points
// straight at its current root, so the second launch's root checks read one
// or two parents (no union runs concurrently here).
template <typename T>
__global__ void __launch_bounds__(256) k_cf_compress(ForceArgs<T> a) {
  const uint32_t nc = a.n_cells[0];
  for (uint32_t id = blockIdx.x * blockDim.x + threadIdx.x; id < nc; id += gridDim.x * blockDim.x) {
    uint32_t budget = kLinkBudget;
    const int m = a.cmin[id];
    const int r = uf_root(a.parent, m, budget);
    if (r >= 0 && r != m) __hip_atomic_store(a.parent + m, r, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// Merging: per cell, its points' sums go to the group root in one set of
// atomics.  Without merging (or for points in no cell): per point.
template <typename T>
__global__ void __launch_bounds__(256) k_cf_sum(ForceArgs<T> a) {
  const uint32_t cnt = cf_count(a);
  const uint32_t nc = (a.scale > T(0)) ? a.n_cells[0] : 0u;
  const size_t C = (size_t)a.ccap;
  // cells: the group root, and the cell's sums (at its smallest contact,
  // which no other cell adds to unless it is the root) added there
  for (uint32_t id = blockIdx.x * blockDim.x + threadIdx.x; id < nc; id += gridDim.x * blockDim.x) {
    uint32_t budget = kLinkBudget;
    const int mn = a.cmin[id];
    int r = uf_root(a.parent, mn, budget);
    if (r < 0) {
      atomicOr(a.status, DEM_DEV_QUEUE_OVERFLOW);
      r = mn;
    }
    a.root[id] = r;
    if (r != mn) {
#pragma unroll
      for (int k = 0; k < 7; ++k) unsafeAtomicAdd(a.acc + (size_t)k * C + r, a.acc[(size_t)k * C + mn]);
    }
  }
  // points in no cell (no merging, or skipped): their own groups
  for (uint32_t c = blockIdx.x * blockDim.x + threadIdx.x; c < cnt; c += gridDim.x * blockDim.x) {
    if (a.pcell[c] >= 0 || !cf_valid(a, c)) continue;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      a.acc[(size_t)d * C + c] = (double)a.x[(size_t)d * C + c];
      a.acc[(size_t)(3 + d) * C + c] = (double)a.n[(size_t)d * C + c];
    }
    a.acc[(size_t)6 * C + c] = 1.0;
  }
}

// Group root of contact c: its cell's, or itself outside any cell.
template <typename T>
__device__ __forceinline__ int cf_root_of(const ForceArgs<T>& a, uint32_t c) {
  const int id = a.pcell[c];
  return id >= 0 ? a.root[id] : (int)c;
}

template <typename T>
__global__ void __launch_bounds__(256) k_cf_emit(ForceArgs<T> a) {
  const uint32_t cnt = cf_count(a);
  for (uint32_t base = blockIdx.x * blockDim.x; base < cnt; base += gridDim.x * blockDim.x) {
    const uint32_t c = base + threadIdx.x;
    const bool is_root = c < cnt && cf_valid(a, c) && cf_root_of(a, c) == (int)c;
    uint32_t ok;
    const uint32_t slot = wave_append(is_root, a.ocount, ok);
    if (!is_root) continue;
    a.mslot[c] = (int32_t)slot;
    if (!ok || slot >= (uint64_t)a.ocap) {
      atomicOr(a.status, DEM_DEV_CONTACT_OVERFLOW);
      continue;
    }
    const double m = a.acc[(size_t)6 * a.ccap + c];
    double xm[3], nm[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      xm[k] = a.acc[(size_t)k * a.ccap + c] / m;
      nm[k] = a.acc[(size_t)(3 + k) * a.ccap + c] / m;
    }
    const int pi = a.pi[c], pj = a.pj[c];
    const double ln = sqrt(nm[0] * nm[0] + nm[1] * nm[1] + nm[2] * nm[2]);
    const double ei = (double)a.teps[a.ti[c]];
    const double mi = (double)a.mass[pi], mj = (double)a.mass[pj];
    // F = n/|n| K_s (1 - |n|/eps_i) sqrt(1 / (1/M_i + 1/M_j)); no direction for n = 0
    const double mag = ln > 0.0 ? (double)a.k_s * (1.0 - ln / ei) * sqrt(1.0 / (1.0 / mi + 1.0 / mj)) / ln : 0.0;
    double f[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) f[k] = mag * nm[k];
    a.opi[slot] = pi;
    a.opj[slot] = pj;
    a.omem[slot] = (int32_t)m;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      a.ox[(size_t)k * a.ocap + slot] = (T)xm[k];
      a.on[(size_t)k * a.ocap + slot] = (T)nm[k];
      a.of[(size_t)k * a.ocap + slot] = (T)f[k];
    }
    const size_t P = (size_t)a.n_particles;
    if (a.force) {
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        atomic_add_t(a.force + k * P + pi, (T)f[k]);
        atomic_add_t(a.force + k * P + pj, (T)(-f[k]));
      }
    }
    if (a.torque) {
      // (x - centre) x force, for both particles
      double ri[3], rj[3];
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        ri[k] = xm[k] - (double)a.centre[k * P + pi];
        rj[k] = xm[k] - (double)a.centre[k * P + pj];
      }
      const double ti[3] = {ri[1] * f[2] - ri[2] * f[1], ri[2] * f[0] - ri[0] * f[2], ri[0] * f[1] - ri[1] * f[0]};
      const double tj[3] = {-(rj[1] * f[2] - rj[2] * f[1]), -(rj[2] * f[0] - rj[0] * f[2]),
                            -(rj[0] * f[1] - rj[1] * f[0])};
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        atomic_add_t(a.torque + k * P + pi, (T)ti[k]);
        atomic_add_t(a.torque + k * P + pj, (T)tj[k]);
      }
    }
  }
}

template <typename T>
__global__ void __launch_bounds__(256) k_cf_group(ForceArgs<T> a) {
  const uint32_t cnt = cf_count(a);
  for (uint32_t c = blockIdx.x * blockDim.x + threadIdx.x; c < cnt; c += gridDim.x * blockDim.x)
    a.group[c] = cf_valid(a, c) ? a.mslot[cf_root_of(a, c)] : -1;
}

__global__ void k_cf_reset(uint32_t* ocount) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *ocount = 0;
}

// ------------------------------------------------------------------ host
IterParams make_iter(const dem_params& p) {
  IterParams ip;
  ip.n_iter = p.n_iter;
  double rho = p.alpha_it_ratio;
  ip.nkappa = (float)(-rho / (rho + 1.0));
  ip.init_centroid = p.init_centroid;
  return ip;
}

bool scene_ok(const dem_scene* s) {
  if (!s) return false;
  if (s->precision != DEM_F32 && s->precision != DEM_F64) return false;
  if (s->n_verts <= 0 || s->n_tris <= 0 || s->n_particles <= 0) return false;
  if (s->n_levels_max < 1 || s->n_levels_max > DEM_MAX_LEVELS) return false;
  if (!s->verts || !s->tri_verts || !s->child_begin || !s->child_count || !s->tri_particle ||
      !s->tri_eps || !s->root_begin || !s->root_count || !s->fine_begin || !s->fine_count)
    return false;
  if (s->fine_parents) {
    if (s->fine_parent_begin[0] != 0) return false;
    for (int d = 0; d < s->n_levels_max; ++d)
      if (s->fine_parent_begin[d + 1] < s->fine_parent_begin[d] ||
          s->fine_parent_begin[d + 1] > s->n_tris)
        return false;
  }
  return true;
}

bool params_ok(const dem_params& p) {
  if (p.mode != DEM_MODE_FLAT && p.mode != DEM_MODE_HIER) return false;
  if (p.n_iter < 0 || p.n_iter > 8) return false;
  if (!(p.omega > 0.0f) || !(p.alpha_reg_rel >= 0.0f) || !(p.alpha_it_ratio > 0.0f)) return false;
  if (p.block != 64 && p.block != 128 && p.block != 256) return false;
  if (p.batch_items < 1 || p.batch_items > p.block) return false;  // one item per thread
  if (p.flat_tile_i < 64 || p.flat_tile_i > 1024 || p.flat_tile_i % 64) return false;
  if (p.flat_tile_j < 1 || p.flat_tile_j > 64) return false;
  if (p.seed_chunk < 1 || p.seed_chunk > 16) return false;
  if (p.queue_capacity < kSeg || p.queue_capacity > (int64_t)0xFFFFFFFF) return false;
  if (p.near_capacity < kSeg || p.near_capacity > (int64_t)0xFFFFFFFF) return false;
  // every block count covers all kSeg segments (blocks of XCD x consume segment x)
  if (p.grid < 0 || (p.grid > 0 && p.grid < kSeg)) return false;
  if (p.frontier_grid < 0 || p.frontier_grid > kFrMaxGrid) return false;
  if (p.half_depths < 0 || p.half_depths > DEM_MAX_LEVELS) return false;
  for (int d = 0; d < DEM_MAX_LEVELS; ++d) {
    if (p.level_grid[d] < 0 || (p.level_grid[d] > 0 && p.level_grid[d] < kSeg)) return false;
    if (p.level_batch[d] < 0 || p.level_batch[d] > p.block) return false;  // one item per thread
  }
  if (p.n_events < 0 || (p.n_events > 0 && !p.events)) return false;
  if (p.persistent != 0 && p.persistent != 1) return false;
  if (p.persistent && p.block != 256) return false;  // the persistent descent runs 256-thread blocks
  if (p.persistent_spins < 0) return false;
  return true;
}

// The Newton iteration count is a template parameter so the iteration is
// fully unrolled; counts 0..8 are instantiated.
template <typename T, int BLOCK, bool HALF>
void launch_level_h(int n_iter, dim3 g, hipStream_t st, const SoupRec<T>* soup, const LevelArgs& la) {
  switch (n_iter) {
#define DEM_CASE(N) case N: hipLaunchKernelGGL((k_level<T, N, BLOCK, HALF>), g, dim3(BLOCK), 0, st, soup, la); break;
    DEM_CASE(0) DEM_CASE(1) DEM_CASE(2) DEM_CASE(3) DEM_CASE(4) DEM_CASE(5) DEM_CASE(6) DEM_CASE(7) DEM_CASE(8)
#undef DEM_CASE
  }
}

// The half-precision iteration is a separate instantiation (FP32 only), so
// that the FP32 kernel keeps its own register allocation.
template <typename T, int BLOCK>
void launch_level_b(int n_iter, dim3 g, hipStream_t st, const SoupRec<T>* soup, const LevelArgs& la) {
  if constexpr (sizeof(T) == 4) {
    if (la.half) {
      launch_level_h<T, BLOCK, true>(n_iter, g, st, soup, la);
      return;
    }
  }
  launch_level_h<T, BLOCK, false>(n_iter, g, st, soup, la);
}

// The deepest depth's kernel without the surrogate-survivor path (256-thread
// blocks, full-precision iteration; other shapes take the general kernel).
template <typename T>
void launch_level_leaf(int n_iter, dim3 g, hipStream_t st, const SoupRec<T>* soup, const LevelArgs& la) {
  switch (n_iter) {
#define DEM_CASE(N) case N: hipLaunchKernelGGL((k_level<T, N, 256, false, true>), g, dim3(256), 0, st, soup, la); break;
    DEM_CASE(0) DEM_CASE(1) DEM_CASE(2) DEM_CASE(3) DEM_CASE(4) DEM_CASE(5) DEM_CASE(6) DEM_CASE(7) DEM_CASE(8)
#undef DEM_CASE
  }
}

template <typename T>
void launch_level(int n_iter, dim3 g, dim3 b, hipStream_t st, const SoupRec<T>* soup, const LevelArgs& la,
                  bool deepest = false) {
  if (deepest && b.x == 256 && !la.half) launch_level_leaf<T>(n_iter, g, st, soup, la);
  else if (b.x == 64) launch_level_b<T, 64>(n_iter, g, st, soup, la);
  else if (b.x == 128) launch_level_b<T, 128>(n_iter, g, st, soup, la);
  else launch_level_b<T, 256>(n_iter, g, st, soup, la);
}

// Resident blocks of the persistent descent on the current device (its grid):
// the kernel's occupancy per compute unit times the compute units.  0 if the
// runtime cannot tell.
template <typename T, int N, bool HALF>
int descent_grid() {
  static int cached = -1;
  if (cached < 0) {
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(k_descent<T, N, 256, HALF>),
                                                     256, 0) != hipSuccess)
      return 0;
    cached = per_cu * cus;
  }
  return cached;
}

template <typename T, bool HALF>
dem_status launch_descent_h(int n_iter, hipStream_t st, const SoupRec<T>* soup, const DescentArgs<T>& d) {
  switch (n_iter) {
#define DEM_CASE(N)                                                                              \
  case N: {                                                                                      \
    const int g = descent_grid<T, N, HALF>();                                                    \
    if (g < kSeg) return DEM_ERR_HIP;                                                            \
    hipLaunchKernelGGL((k_descent<T, N, 256, HALF>), dim3(g), dim3(256), 0, st, soup, d);       \
    break;                                                                                       \
  }
    DEM_CASE(0) DEM_CASE(1) DEM_CASE(2) DEM_CASE(3) DEM_CASE(4) DEM_CASE(5) DEM_CASE(6) DEM_CASE(7) DEM_CASE(8)
#undef DEM_CASE
  }
  return DEM_OK;
}

template <typename T>
dem_status launch_descent(int n_iter, bool half, hipStream_t st, const SoupRec<T>* soup, const DescentArgs<T>& d) {
  if constexpr (sizeof(T) == 4) {
    if (half) return launch_descent_h<T, true>(n_iter, st, soup, d);
  }
  return launch_descent_h<T, false>(n_iter, st, soup, d);
}

template <typename T>
void launch_flat(int n_iter, dim3 g, dim3 b, hipStream_t st, const SoupRec<T>* soup, const LevelArgs& la) {
  switch (n_iter) {
#define DEM_CASE(N) case N: hipLaunchKernelGGL((k_flat<T, N, 64>), g, b, 0, st, soup, la); break;
    DEM_CASE(0) DEM_CASE(1) DEM_CASE(2) DEM_CASE(3) DEM_CASE(4) DEM_CASE(5) DEM_CASE(6) DEM_CASE(7) DEM_CASE(8)
#undef DEM_CASE
  }
}

template <typename T, bool FR>
void launch_near_certify(int n_iter, dim3 g, dim3 b, hipStream_t st, const SoupRec<T>* soup, const NearArgs& na) {
  switch (n_iter) {
#define DEM_CASE(N) case N: hipLaunchKernelGGL((k_near<T, N, true, FR>), g, b, 0, st, soup, na); break;
    DEM_CASE(0) DEM_CASE(1) DEM_CASE(2) DEM_CASE(3) DEM_CASE(4) DEM_CASE(5) DEM_CASE(6) DEM_CASE(7) DEM_CASE(8)
#undef DEM_CASE
  }
}

template <typename T>
dem_status run_find(const dem_scene* s, const int32_t* pairs, int n_pairs, const dem_params& p,
                    const dem_contacts* out, void* ws, const WsLayout& L, dem_stats* stats,
                    uint32_t* status, double* energy, hipStream_t st) {
  char* base = static_cast<char*>(ws);
  Counters* ctr = reinterpret_cast<Counters*>(base + L.ctr);
  SoupRec<T>* soup = reinterpret_cast<SoupRec<T>*>(base + L.soup);
  int4* q[2] = {reinterpret_cast<int4*>(base + L.qa), reinterpret_cast<int4*>(base + L.qb)};
  int2* nearl = reinterpret_cast<int2*>(base + L.near_);
  const int grid = p.grid > 0 ? p.grid : 2048;
  int n_launch = 0;
  auto mark = [&]() {
    if (p.events && n_launch < p.n_events)
      (void)hipEventRecord(reinterpret_cast<hipEvent_t>(p.events[n_launch]), st);
    ++n_launch;
  };
  mark();
  hipLaunchKernelGGL(k_reset, dim3(1), dim3(256), 0, st, ctr, stats, status, out->count, energy);
  mark();
  FlatArgs<T> fa{};
  fa.verts = static_cast<const T*>(s->verts);
  fa.n_verts = s->n_verts;
  fa.tv = s->tri_verts;
  fa.n_tris = s->n_tris;
  fa.cbeg = s->child_begin;
  fa.ccnt = s->child_count;
  fa.tpart = s->tri_particle;
  fa.teps = static_cast<const T*>(s->tri_eps);
  fa.pose = static_cast<const T*>(s->pose);
  fa.areg_rel = T(p.alpha_reg_rel);
  fa.omega = T(p.omega);
  fa.root_begin = s->root_begin;
  fa.root_count = s->root_count;
  fa.fine_begin = s->fine_begin;
  fa.soup = soup;
  fa.mark = reinterpret_cast<uint8_t*>(base + L.mark);
  fa.lazy = p.mode == DEM_MODE_HIER && s->fine_parents != nullptr;
  fa.status = status;
  fa.fine_part = stats ? &ctr->fine_part[0][0] : nullptr;
  hipLaunchKernelGGL(k_flatten<T>, dim3((s->n_tris + kFlatBlock - 1) / kFlatBlock), dim3(kFlatBlock), 0, st, fa);
  mark();
  // per-segment capacities
  const int64_t qseg = p.queue_capacity / kSeg, nseg = p.near_capacity / kSeg;
  LevelArgs la{};
  la.qcap = qseg;
  la.near_ = nearl;
  la.near_tail = ctr->near_tail;
  la.ncap = nseg;
  la.stats = stats;
  la.part = stats ? ctr->stat_part : nullptr;
  la.status = status;
  la.dense = p.dense_distance;
  la.batch = p.batch_items;
  la.mark = nullptr;
  la.ip = make_iter(p);
  if (n_pairs > 0 && p.mode == DEM_MODE_HIER && p.persistent) {
    DescentArgs<T> d{};
    d.a = la;
    d.a.mark = fa.lazy ? fa.mark : nullptr;
    d.q0 = q[0];
    d.q1 = q[1];
    d.ctr = ctr;
    d.n_levels = s->n_levels_max;
    d.half_depths = s->precision == DEM_F32 ? p.half_depths : 0;
    d.spin_limit = p.persistent_spins > 0 ? (uint32_t)p.persistent_spins : kBarrierSpins;
    for (int lev = 0; lev < DEM_MAX_LEVELS; ++lev)
      d.batch[lev] = p.level_batch[lev] > 0 ? p.level_batch[lev] : p.batch_items;
    d.pairs = pairs;
    d.n_pairs = n_pairs;
    d.rbeg = s->root_begin;
    d.rcnt = s->root_count;
    d.seed_chunk = p.seed_chunk;
    d.f = fa;
    d.fine_parents = fa.lazy ? s->fine_parents : nullptr;
    for (int lev = 0; lev <= DEM_MAX_LEVELS; ++lev) d.fine_parent_begin[lev] = fa.lazy ? s->fine_parent_begin[lev] : 0;
    const dem_status r = launch_descent<T>(p.n_iter, d.half_depths > 0, st, soup, d);
    if (r != DEM_OK) return r;
    mark();
  } else if (n_pairs > 0) {
    if (p.mode == DEM_MODE_HIER) {
      hipLaunchKernelGGL(k_seed, dim3(n_pairs), dim3(256), 0, st, pairs, n_pairs, s->root_begin,
                         s->root_count, p.seed_chunk, p.seed_chunk, q[0], ctr->tail[0], qseg, status);
      mark();
      for (int lev = 0; lev < s->n_levels_max; ++lev) {
        la.qin = q[lev & 1];
        la.tail_in = ctr->tail[lev];
        la.qout = q[(lev + 1) & 1];
        la.tail_out = ctr->tail[lev + 1];
        la.depth = lev;
        la.deepest = lev == s->n_levels_max - 1;
        la.batch = p.level_batch[lev] > 0 ? p.level_batch[lev] : p.batch_items;
        la.mark = fa.lazy ? fa.mark : nullptr;
        la.half = s->precision == DEM_F32 && lev < p.half_depths;
        const int g = p.level_grid[lev] > 0 ? p.level_grid[lev] : grid;
        launch_level<T>(p.n_iter, dim3(g), dim3(p.block), st, soup, la, lev == s->n_levels_max - 1);
        mark();
        // lazy flattening: children of this depth's surviving parents
        const int f0 = fa.lazy ? s->fine_parent_begin[lev] : 0;
        const int nf = fa.lazy ? s->fine_parent_begin[lev + 1] - f0 : 0;
        if (nf > 0)
          hipLaunchKernelGGL(k_fine<T>, dim3(std::min((nf + kFlatBlock - 1) / kFlatBlock, 1 << 20)), dim3(kFlatBlock), 0,
                             st, fa, s->fine_parents + f0, nf);
        mark();
      }
    } else {
      hipLaunchKernelGGL(k_seed, dim3(n_pairs), dim3(256), 0, st, pairs, n_pairs, s->fine_begin,
                         s->fine_count, p.flat_tile_i, p.flat_tile_j, q[0], ctr->tail[0], qseg, status);
      mark();
      la.qin = q[0];
      la.tail_in = ctr->tail[0];
      la.qout = q[1];
      la.tail_out = ctr->tail[1];
      la.depth = 0;
      launch_flat<T>(p.n_iter, dim3(grid), dim3(p.flat_tile_i > 256 ? 256 : p.flat_tile_i), st, soup, la);
      mark();
    }
  }
  NearArgs na{};
  na.near_ = nearl;
  na.near_tail = ctr->near_tail;
  na.ncap = nseg;
  na.fb = reinterpret_cast<int2*>(base + L.fb);
  na.fb_tail = ctr->fb_tail;
  na.pi = out->pi; na.pj = out->pj; na.ti = out->ti; na.tj = out->tj;
  na.d = out->d; na.x = out->x; na.n = out->n;
  na.adj = out->adjoint;
  na.count = out->count;
  na.ccap = out->capacity;
  na.dense = p.dense_distance;
  na.k = p.energy_k;
  na.energy = energy;
  na.stats = stats;
  na.part = (stats || energy) ? ctr->stat_part : nullptr;
  na.status = status;
  na.ip = make_iter(p);
  if (p.certify) {
    launch_near_certify<T, false>(p.n_iter, dim3(grid), dim3(p.block), st, soup, na);
    mark();
    // the exact comparison-based pass over what the certificate left
    na.near_ = na.fb;
    na.near_tail = na.fb_tail;
  }
  hipLaunchKernelGGL((k_near<T, 0, false, false>), dim3(grid), dim3(p.block), 0, st, soup, na);
  mark();
  if (stats || energy) {
    hipLaunchKernelGGL(k_fold_stats, dim3(1), dim3(64), 0, st, ctr->stat_part, &ctr->fine_part[0][0],
                       s->n_levels_max, stats, energy);
    mark();
  }
  return hipGetLastError() == hipSuccess ? DEM_OK : DEM_ERR_HIP;
}


// ------------------------------------------------------------------ frontier host side
struct FrLayout {
  WsLayout w;
  size_t meta, cm, part, pcount, total;
};

int fr_grid(const dem_params& p) { return p.frontier_grid > 0 ? p.frontier_grid : 4096; }

FrLayout fr_layout(int precision, int64_t n_tris, int64_t ncap, int64_t fcap, int grid, int64_t n_pairs) {
  FrLayout F;
  F.w = ws_layout(precision, n_tris, kSeg, ncap);  // level queues unused: minimal
  size_t o = F.w.total;
  F.meta = o; o = align_up(o + 4 * (size_t)fcap, 256);
  F.cm = o; o = align_up(o + (size_t)fcap, 256);
  F.part = o; o = align_up(o + 8 * (size_t)(grid + 1), 256);
  F.pcount = o; o = align_up(o + 8 * (size_t)(n_pairs + 1), 256);
  F.total = o;
  return F;
}

bool frontier_ok(const dem_frontier* f) {
  if (!f || !f->leaves[0] || !f->leaves[1] || !f->state || !f->memory) return false;
  if (f->capacity < 1 || f->capacity > (int64_t)0xFFFFFFFF) return false;
  if (f->memory_capacity < 64 || (f->memory_capacity & (f->memory_capacity - 1))) return false;
  if (reinterpret_cast<uintptr_t>(f->leaves[0]) % 16 || reinterpret_cast<uintptr_t>(f->leaves[1]) % 16) return false;
  return true;
}

template <typename T>
void launch_fr_eval(int n_iter, dim3 g, hipStream_t st, const SoupRec<T>* soup, const FrontierArgs& fa) {
  switch (n_iter) {
#define DEM_CASE(N) case N: hipLaunchKernelGGL((k_fr_eval<T, N, false>), g, dim3(kFrBlock), 0, st, soup, fa); break;
    DEM_CASE(0) DEM_CASE(1) DEM_CASE(2) DEM_CASE(3) DEM_CASE(4) DEM_CASE(5) DEM_CASE(6) DEM_CASE(7) DEM_CASE(8)
#undef DEM_CASE
  }
}

template <typename T>
dem_status run_frontier_step(const dem_scene* s, const dem_params& p, const dem_frontier* f,
                             const dem_contacts* out, void* ws, const FrLayout& FL, dem_stats* stats,
                             uint32_t* status, double* energy, hipStream_t st) {
  char* base = static_cast<char*>(ws);
  Counters* ctr = reinterpret_cast<Counters*>(base + FL.w.ctr);
  SoupRec<T>* soup = reinterpret_cast<SoupRec<T>*>(base + FL.w.soup);
  const int grid = fr_grid(p);                 // per-leaf kernels
  const int ngrid = p.grid > 0 ? p.grid : 2048;  // near-pair kernels, as in the descent
  int n_launch = 0;
  auto mark = [&]() {
    if (p.events && n_launch < p.n_events)
      (void)hipEventRecord(reinterpret_cast<hipEvent_t>(p.events[n_launch]), st);
    ++n_launch;
  };
  mark();
  hipLaunchKernelGGL(k_reset, dim3(1), dim3(256), 0, st, ctr, stats, status, out->count, energy);
  mark();
  FlatArgs<T> fl{};
  fl.verts = static_cast<const T*>(s->verts);
  fl.n_verts = s->n_verts;
  fl.tv = s->tri_verts;
  fl.n_tris = s->n_tris;
  fl.cbeg = s->child_begin;
  fl.ccnt = s->child_count;
  fl.tpart = s->tri_particle;
  fl.teps = static_cast<const T*>(s->tri_eps);
  fl.pose = static_cast<const T*>(s->pose);
  fl.areg_rel = T(p.alpha_reg_rel);
  fl.omega = T(p.omega);
  fl.root_begin = s->root_begin;
  fl.root_count = s->root_count;
  fl.fine_begin = s->fine_begin;
  fl.soup = soup;
  fl.mark = reinterpret_cast<uint8_t*>(base + FL.w.mark);
  fl.lazy = 0;  // leaves may sit at any depth: every record is written
  fl.status = status;
  hipLaunchKernelGGL(k_flatten<T>, dim3((s->n_tris + kFlatBlock - 1) / kFlatBlock), dim3(kFlatBlock), 0, st, fl);
  mark();
  const int64_t nseg = p.near_capacity / kSeg;
  FrontierArgs fa{};
  fa.buf0 = reinterpret_cast<int4*>(f->leaves[0]);
  fa.buf1 = reinterpret_cast<int4*>(f->leaves[1]);
  fa.state = f->state;
  fa.cap = f->capacity;
  fa.mem = reinterpret_cast<unsigned long long*>(f->memory);
  fa.mem_mask = (uint64_t)f->memory_capacity - 1;
  fa.meta = reinterpret_cast<uint32_t*>(base + FL.meta);
  fa.cm = reinterpret_cast<uint8_t*>(base + FL.cm);
  fa.part = reinterpret_cast<unsigned long long*>(base + FL.part);
  fa.tri_parent = s->tri_parent;
  fa.tri_depth = s->tri_depth;
  fa.cbeg = s->child_begin;
  fa.ccnt = s->child_count;
  fa.n_tris = s->n_tris;
  fa.ctr = ctr;
  fa.near_ = reinterpret_cast<int2*>(base + FL.w.near_);
  fa.near_tail = ctr->near_tail;
  fa.ncap = nseg;
  fa.stats = stats;
  fa.spart = stats ? ctr->stat_part : nullptr;
  fa.status = status;
  fa.ip = make_iter(p);
  if (p.prune_exact) hipLaunchKernelGGL((k_fr_eval<T, 0, true>), dim3(grid), dim3(kFrBlock), 0, st, soup, fa);
  else launch_fr_eval<T>(p.n_iter, dim3(grid), st, soup, fa);
  mark();
  NearArgs na{};
  na.near_ = fa.near_;
  na.near_tail = ctr->near_tail;
  na.ncap = nseg;
  na.fb = reinterpret_cast<int2*>(base + FL.w.fb);
  na.fb_tail = ctr->fb_tail;
  na.pi = out->pi; na.pj = out->pj; na.ti = out->ti; na.tj = out->tj;
  na.d = out->d; na.x = out->x; na.n = out->n;
  na.adj = out->adjoint;
  na.count = out->count;
  na.ccap = out->capacity;
  na.dense = 0;
  na.k = p.energy_k;
  na.energy = energy;
  na.stats = stats;
  na.status = status;
  na.ip = make_iter(p);
  na.fr_buf0 = fa.buf0;
  na.fr_buf1 = fa.buf1;
  na.fr_state = f->state;
  na.fr_meta = reinterpret_cast<uint8_t*>(fa.meta);
  na.part = (stats || energy) ? ctr->stat_part : nullptr;  // summed by k_fold_stats at the end
  if (p.certify) {
    launch_near_certify<T, true>(p.n_iter, dim3(ngrid), dim3(p.block), st, soup, na);
    mark();
    na.near_ = na.fb;
    na.near_tail = na.fb_tail;
  }
  hipLaunchKernelGGL((k_near<T, 0, false, true>), dim3(ngrid), dim3(p.block), 0, st, soup, na);
  mark();
  hipLaunchKernelGGL(k_fr_group, dim3(grid), dim3(kFrBlock), 0, st, fa);
  mark();
  hipLaunchKernelGGL(k_fr_scan, dim3(1), dim3(kScanThreads), 0, st, fa, (uint32_t)grid);
  mark();
  hipLaunchKernelGGL(k_fr_emit, dim3(grid), dim3(kFrBlock), 0, st, fa);
  mark();
  hipLaunchKernelGGL(k_fr_finish, dim3(1), dim3(64), 0, st, fa);
  mark();
  if (na.part)
    hipLaunchKernelGGL(k_fold_stats, dim3(1), dim3(64), 0, st, ctr->stat_part, &ctr->fine_part[0][0],
                       DEM_MAX_LEVELS, stats, energy);
  mark();  // (the fold's slot, empty without statistics and energy)
  return hipGetLastError() == hipSuccess ? DEM_OK : DEM_ERR_HIP;
}


// ------------------------------------------------------------------ contact forces host side
struct CfLayout {
  uint64_t table;
  size_t keys, scnt, sid, counters, coff, ccnt, cfill, cmin, crec, pcell, order, pts, parent, root, mslot, acc,
      total;
};

CfLayout cf_layout(int64_t cap) {
  CfLayout L;
  const uint64_t want = std::max<uint64_t>(1024, 2 * (uint64_t)cap);
  L.table = 1;
  while (L.table < want) L.table <<= 1;
  const size_t T = L.table, C = (size_t)cap;
  size_t o = 0;
  L.keys = o; o = align_up(o + 8 * T, 256);
  L.scnt = o; o = align_up(o + 4 * T, 256);
  L.sid = o; o = align_up(o + 4 * T, 256);
  L.counters = o; o = align_up(o + 8, 256);
  L.coff = o; o = align_up(o + 4 * C, 256);
  L.ccnt = o; o = align_up(o + 4 * C, 256);
  L.cfill = o; o = align_up(o + 4 * C, 256);
  L.cmin = o; o = align_up(o + 4 * C, 256);
  L.crec = o; o = align_up(o + sizeof(CellRec<double>) * C, 256);
  L.pcell = o; o = align_up(o + 4 * C, 256);
  L.order = o; o = align_up(o + 4 * C, 256);
  L.pts = o; o = align_up(o + 8 * 8 * C, 256);  // room for FP64
  L.parent = o; o = align_up(o + 4 * C, 256);
  L.root = o; o = align_up(o + 4 * C, 256);
  L.mslot = o; o = align_up(o + 4 * C, 256);
  L.acc = o; o = align_up(o + 8 * 7 * C, 256);
  L.total = o;
  return L;
}

template <typename T>
dem_status run_forces(const dem_scene* s, const dem_contacts* c, const void* mass, const void* centre, double k_s,
                      double scale, const dem_merged* out, int32_t* group, void* force, void* torque, void* ws,
                      const CfLayout& L, uint32_t* status, hipStream_t st) {
  char* base = static_cast<char*>(ws);
  ForceArgs<T> a;
  a.pi = c->pi; a.pj = c->pj; a.ti = c->ti; a.tj = c->tj;
  a.x = static_cast<const T*>(c->x);
  a.n = static_cast<const T*>(c->n);
  a.ccap = c->capacity;
  a.ccount = c->count;
  a.teps = static_cast<const T*>(s->tri_eps);
  a.n_tris = s->n_tris;
  a.scale = (T)scale;
  a.keys = reinterpret_cast<unsigned long long*>(base + L.keys);
  a.scnt = reinterpret_cast<uint32_t*>(base + L.scnt);
  a.sid = reinterpret_cast<int32_t*>(base + L.sid);
  a.tmask = L.table - 1;
  a.n_cells = reinterpret_cast<uint32_t*>(base + L.counters);
  a.coff = reinterpret_cast<uint32_t*>(base + L.coff);
  a.ccnt = reinterpret_cast<uint32_t*>(base + L.ccnt);
  a.cfill = reinterpret_cast<uint32_t*>(base + L.cfill);
  a.cmin = reinterpret_cast<int32_t*>(base + L.cmin);
  a.crec = reinterpret_cast<CellRec<T>*>(base + L.crec);
  a.pcell = reinterpret_cast<int32_t*>(base + L.pcell);
  a.order = reinterpret_cast<int32_t*>(base + L.order);
  a.pts = reinterpret_cast<T*>(base + L.pts);
  a.parent = reinterpret_cast<int32_t*>(base + L.parent);
  a.root = reinterpret_cast<int32_t*>(base + L.root);
  a.mslot = reinterpret_cast<int32_t*>(base + L.mslot);
  a.acc = reinterpret_cast<double*>(base + L.acc);
  a.mass = static_cast<const T*>(mass);
  a.centre = static_cast<const T*>(centre);
  a.n_particles = s->n_particles;
  a.k_s = (T)k_s;
  a.opi = out->pi; a.opj = out->pj;
  a.ox = static_cast<T*>(out->x);
  a.on = static_cast<T*>(out->n);
  a.of = static_cast<T*>(out->f);
  a.omem = out->members;
  a.ocount = out->count;
  a.ocap = out->capacity;
  a.group = group;
  a.force = static_cast<T*>(force);
  a.torque = static_cast<T*>(torque);
  a.status = status;
  const dim3 g(2048), b(256), gt(4096);
  hipLaunchKernelGGL(k_cf_reset, dim3(1), dim3(64), 0, st, out->count);
  if (c->capacity > 0) {
    const bool merge = scale > 0.0;
    hipLaunchKernelGGL(k_cf_clear<T>, gt, b, 0, st, a, merge ? (uint64_t)L.table : (uint64_t)0);
    hipLaunchKernelGGL(k_cf_insert<T>, g, b, 0, st, a);
    if (merge) {
      hipLaunchKernelGGL(k_cf_range<T>, gt, b, 0, st, a, (uint64_t)L.table);
      hipLaunchKernelGGL(k_cf_place<T>, g, b, 0, st, a);
      hipLaunchKernelGGL(k_cf_cells<T>, g, b, 0, st, a);
      // adjacent cells first: they join most of a patch, so that the distant
      // offsets mostly find both cells in one group already
      hipLaunchKernelGGL(k_cf_link<T>, g, b, 0, st, a, 0, kNbrAdjacent);
      hipLaunchKernelGGL(k_cf_compress<T>, g, b, 0, st, a);
      hipLaunchKernelGGL(k_cf_link<T>, g, b, 0, st, a, kNbrAdjacent, kNbr);
    }
    hipLaunchKernelGGL(k_cf_sum<T>, g, b, 0, st, a);
    hipLaunchKernelGGL(k_cf_emit<T>, g, b, 0, st, a);
    if (group) hipLaunchKernelGGL(k_cf_group<T>, g, b, 0, st, a);
  }
  return hipGetLastError() == hipSuccess ? DEM_OK : DEM_ERR_HIP;
}


// ------------------------------------------------------------------ deterministic order
// dem_sort_contacts: the contacts reordered by (t_i, t_j), the global triangle
// numbers (a contact's triangle pair is unique, so the order is total): a
// counting sort by t_i, with the bucket offsets from a prefix sum over the
// triangles, then every bucket sorted by t_j.  Kernels only, so the call can
// be captured in a graph.  Contacts naming a triangle outside the scene keep
// their relative order after all others (and are flagged).
constexpr uint32_t kSortThreads = 256;
constexpr uint32_t kSortPer = 16;                          // buckets per thread in the scan
constexpr uint32_t kSortChunk = kSortThreads * kSortPer;   // buckets per scan block

struct SortArgs {
  int32_t* pi;
  int32_t* pj;
  int32_t* ti;
  int32_t* tj;
  void* d;
  void* x;
  void* n;
  void* adj;                  // adjoint rows or null
  const uint32_t* count;
  int64_t cap;
  uint32_t n_buckets;         // n_tris + 1 (the last one: invalid triangle numbers)
  uint32_t* hist;             // [n_buckets]: counts, then exclusive offsets
  uint32_t* fill;             // [n_buckets]
  unsigned long long* bsum;   // [scan blocks + 1]
  int32_t* idx;               // [cap]: input contact of every output position
  char* tmp;                  // [cap] records of the reordered fields
  uint32_t* blist;            // [n_buckets]: buckets of two or more contacts
  uint32_t* blist_n;          // their number
  uint32_t* status;
};

struct SortLayout {
  size_t hist, fill, bsum, idx, tmp, blist, total;
  uint32_t n_buckets, n_blocks;
};

__device__ __forceinline__ uint32_t cs_count(const SortArgs& a) {
  return (uint32_t)min((uint64_t)*a.count, (uint64_t)a.cap);
}

__device__ __forceinline__ uint32_t cs_bucket(const SortArgs& a, uint32_t c) {
  const uint32_t t = (uint32_t)a.ti[c];
  return t < a.n_buckets - 1 ? t : a.n_buckets - 1;
}

__global__ void k_cs_clear(SortArgs a) {
  for (uint32_t k = blockIdx.x * blockDim.x + threadIdx.x; k < a.n_buckets; k += gridDim.x * blockDim.x) {
    a.hist[k] = 0;
    a.fill[k] = 0;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) *a.blist_n = 0;
}

// Runs of neighbouring lanes with one bucket (the contacts of one triangle
// come in short runs): the run's first lane counts or reserves for all of it.
struct LaneRun {
  bool lead;      // first lane of its run
  int len;        // run length (at the leader)
  int leader;     // the run's first lane
};

__device__ __forceinline__ LaneRun lane_run(bool act, uint32_t key) {
  const int lane = lane_id();
  const uint32_t prev = __shfl_up(key, 1);
  const bool prev_act = __shfl_up((int)act, 1) != 0;
  LaneRun r;
  r.lead = act && (lane == 0 || !prev_act || prev != key);
  const unsigned long long leaders = __ballot(r.lead), members = __ballot(act);
  const unsigned long long after = lane == 63 ? 0ull : (~0ull << (lane + 1));
  const unsigned long long stops = (leaders | ~members) & after;
  r.len = (stops ? __ffsll((long long)stops) - 1 : 64) - lane;
  const unsigned long long upto = lane == 63 ? ~0ull : ((2ull << lane) - 1ull);
  r.leader = act ? 63 - __clzll((long long)(leaders & upto)) : lane;
  return r;
}

__global__ void k_cs_count(SortArgs a) {
  const uint32_t cnt = cs_count(a);
  for (uint32_t base = blockIdx.x * blockDim.x; base < cnt; base += gridDim.x * blockDim.x) {
    const uint32_t c = base + threadIdx.x;
    const bool act = c < cnt;
    const uint32_t b = act ? cs_bucket(a, c) : 0u;
    if (act && (b == a.n_buckets - 1 || (uint32_t)a.tj[c] >= a.n_buckets - 1)) atomicOr(a.status, DEM_DEV_BAD_TREE);
    const LaneRun r = lane_run(act, b);
    if (r.lead) atomicAdd(a.hist + b, (uint32_t)r.len);
  }
}

// Scan block b covers buckets [b * kSortChunk, ...): thread t its kSortPer
// consecutive buckets.
__global__ void __launch_bounds__(kSortThreads) k_cs_bsum(SortArgs a) {
  __shared__ unsigned long long red[kSortThreads / kWave];
  const uint32_t lo = blockIdx.x * kSortChunk + threadIdx.x * kSortPer;
  unsigned long long s = 0;
  for (uint32_t k = 0; k < kSortPer; ++k)
    if (lo + k < a.n_buckets) s += a.hist[lo + k];
  s = wave_sum_u64(s);
  if (lane_id() == 0) red[threadIdx.x / kWave] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long t = 0;
    for (uint32_t w = 0; w < kSortThreads / kWave; ++w) t += red[w];
    a.bsum[blockIdx.x] = t;
  }
}

__global__ void __launch_bounds__(kScanThreads) k_cs_top(SortArgs a, uint32_t n_blocks) {
  block_scan_u64(a.bsum, n_blocks);
}

__global__ void __launch_bounds__(kSortThreads) k_cs_local(SortArgs a) {
  __shared__ unsigned long long wsum[kSortThreads / kWave];
  const uint32_t lo = blockIdx.x * kSortChunk + threadIdx.x * kSortPer;
  uint32_t v[kSortPer];
  unsigned long long s = 0;
#pragma unroll
  for (uint32_t k = 0; k < kSortPer; ++k) {
    v[k] = lo + k < a.n_buckets ? a.hist[lo + k] : 0u;
    s += v[k];
  }
  const int lane = lane_id(), wid = threadIdx.x / kWave;
  unsigned long long x = s;
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    const unsigned long long y = __shfl_up(x, o);
    if (lane >= o) x += y;
  }
  if (lane == kWave - 1) wsum[wid] = x;
  __syncthreads();
  unsigned long long before = a.bsum[blockIdx.x];
  for (int w = 0; w < wid; ++w) before += wsum[w];
  unsigned long long run = before + x - s;
#pragma unroll
  for (uint32_t k = 0; k < kSortPer; ++k) {
    if (lo + k < a.n_buckets) a.hist[lo + k] = (uint32_t)run;
    run += v[k];
  }
}

__global__ void k_cs_scatter(SortArgs a) {
  const uint32_t cnt = cs_count(a);
  const int lane = lane_id();
  for (uint32_t base = blockIdx.x * blockDim.x; base < cnt; base += gridDim.x * blockDim.x) {
    const uint32_t c = base + threadIdx.x;
    const bool act = c < cnt;
    const uint32_t b = act ? cs_bucket(a, c) : 0u;
    const LaneRun r = lane_run(act, b);
    uint32_t pos = 0;
    if (r.lead) pos = a.hist[b] + atomicAdd(a.fill + b, (uint32_t)r.len);
    pos = __shfl(pos, r.leader) + (uint32_t)(lane - r.leader);
    if (act) a.idx[pos] = (int32_t)c;
  }
}

// Every bucket by t_j (the last bucket, of invalid triangle numbers, by
// input position), by ranks: a contact's position is the number of smaller
// keys in its bucket (the keys of a bucket are distinct).  Buckets inside
// one window of 64 output positions (most) are ranked by k_cs_small; the
// rest are listed and ranked one per wave by k_cs_bucket.
constexpr uint32_t kBucketLds = 512;

__device__ __forceinline__ long long cs_key(const SortArgs& a, bool by_input, int32_t c) {
  return by_input ? (long long)c : (long long)a.tj[c];
}

// A bucket of two or more contacts whose output range lies inside one
// aligned window of 64 positions is ranked by k_cs_small.
__device__ __forceinline__ bool cs_in_window(uint32_t lo, uint32_t m) {
  return (lo / kWave) == ((lo + m - 1) / kWave);
}

// The other buckets to sort (two or more contacts, across a window boundary,
// or of invalid triangle numbers), listed so that the sorting waves share
// them evenly (contacts cluster in the triangle numbering).
__global__ void k_cs_list(SortArgs a) {
  for (uint32_t base = blockIdx.x * blockDim.x; base < a.n_buckets; base += gridDim.x * blockDim.x) {
    const uint32_t b = base + threadIdx.x;
    const uint32_t m = b < a.n_buckets ? a.fill[b] : 0u;
    const bool need = m >= 2 && (b == a.n_buckets - 1 || !cs_in_window(a.hist[b], m));
    uint32_t ok;
    const uint32_t slot = wave_append(need, a.blist_n, ok);
    if (need && ok && slot < a.n_buckets) a.blist[slot] = b;
  }
}

// The buckets inside one window (most: a triangle has a few contacts), by
// the window's wave: lane p holds output position p's contact, reads its
// bucket's range from the offsets, and counts the smaller keys among the
// bucket's lanes (keys through the wave's LDS slice).  Every lane reads
// before any lane writes, and a window's writes stay inside it.
__global__ void __launch_bounds__(256) k_cs_small(SortArgs a) {
  __shared__ long long skey[256 / kWave][kWave];
  const uint32_t cnt = cs_count(a);
  const int lane = lane_id(), w = threadIdx.x / kWave;
  for (uint32_t base = blockIdx.x * blockDim.x; base < cnt; base += gridDim.x * blockDim.x) {
    const uint32_t p = base + threadIdx.x;
    const uint32_t W = p - (uint32_t)lane;  // the window (base is a multiple of the block)
    const bool act = p < cnt;
    int32_t v = 0;
    uint32_t b = 0, lo = 0, m = 0;
    long long kk = LLONG_MAX;
    if (act) {
      v = a.idx[p];
      b = cs_bucket(a, (uint32_t)v);
      lo = a.hist[b];
      m = a.fill[b];
      kk = (long long)a.tj[v];
    }
    const bool mine = act && b != a.n_buckets - 1 && m >= 2 && cs_in_window(lo, m);
    skey[w][lane] = kk;
    __builtin_amdgcn_wave_barrier();
    uint32_t rank = 0;
    if (mine)
      for (uint32_t j = lo - W; j < lo - W + m; ++j) rank += skey[w][j] < kk ? 1u : 0u;
    __builtin_amdgcn_wave_barrier();
    if (mine) a.idx[lo + rank] = v;
    __builtin_amdgcn_wave_barrier();
  }
}

// One wave per listed bucket.  Up to kBucketLds contacts: keys and contacts
// into the wave's LDS slice first, so that every read of the bucket precedes
// the writes and each contact is placed directly at its rank; longer
// buckets 64 contacts at a time through the staging area.
__global__ void __launch_bounds__(256) k_cs_bucket(SortArgs a) {
  __shared__ long long skey[256 / kWave][kBucketLds];
  __shared__ int32_t sval[256 / kWave][kBucketLds];
  const uint32_t lane = (uint32_t)lane_id();
  const int w = threadIdx.x / kWave;
  int32_t* stage = reinterpret_cast<int32_t*>(a.tmp);  // free until the gather
  const uint32_t nl = min(*a.blist_n, a.n_buckets);
  const uint32_t nw = gridDim.x * (blockDim.x / kWave);
  for (uint32_t q = blockIdx.x * (blockDim.x / kWave) + (uint32_t)w; q < nl; q += nw) {
    const uint32_t bw = a.blist[q];
    const uint32_t mw = a.fill[bw], low = a.hist[bw];
    const bool by_input = bw == a.n_buckets - 1;
    int32_t* e = a.idx + low;
    if (mw <= (uint32_t)kWave) {
      // one contact per lane: every read of the bucket precedes the writes
      const bool act = lane < mw;
      const int32_t v = act ? e[lane] : 0;
      const long long kk = act ? cs_key(a, by_input, v) : LLONG_MAX;
      skey[w][lane] = kk;
      __builtin_amdgcn_wave_barrier();
      uint32_t rank = 0;
      for (uint32_t j = 0; j < mw; ++j) rank += skey[w][j] < kk ? 1u : 0u;
      __builtin_amdgcn_wave_barrier();
      if (act) e[rank] = v;
      continue;
    }
    if (mw <= kBucketLds) {
      for (uint32_t r = lane; r < mw; r += kWave) {
        const int32_t v = e[r];
        sval[w][r] = v;
        skey[w][r] = cs_key(a, by_input, v);
      }
      __builtin_amdgcn_wave_barrier();
      for (uint32_t r = lane; r < mw; r += kWave) {
        const long long kk = skey[w][r];
        uint32_t rank = 0;
        for (uint32_t j = 0; j < mw; ++j) rank += skey[w][j] < kk ? 1u : 0u;
        e[rank] = sval[w][r];
      }
      __builtin_amdgcn_wave_barrier();
      continue;
    }
    for (uint32_t k0 = 0; k0 < mw; k0 += kWave) {
      const uint32_t k = k0 + lane;
      const bool act = k < mw;
      const int32_t v = act ? e[k] : 0;
      const long long kk = act ? cs_key(a, by_input, v) : LLONG_MAX;
      uint32_t rank = 0;
      for (uint32_t c0 = 0; c0 < mw; c0 += kBucketLds) {
        const uint32_t n = min(kBucketLds, mw - c0);
        for (uint32_t r = lane; r < n; r += kWave) skey[w][r] = cs_key(a, by_input, e[c0 + r]);
        __builtin_amdgcn_wave_barrier();
        for (uint32_t j = 0; j < n; ++j) rank += skey[w][j] < kk ? 1u : 0u;
        __builtin_amdgcn_wave_barrier();
      }
      if (act) stage[low + rank] = v;
    }
    // lanes read back what other lanes placed: device-scope fences
    __threadfence();
    __builtin_amdgcn_wave_barrier();
    for (uint32_t k = lane; k < mw; k += kWave) e[k] = stage[low + k];
    __threadfence();
    __builtin_amdgcn_wave_barrier();
  }
}

template <typename T>
struct SortRec {
  int32_t pi, pj, ti, tj;
  T d, x[3], n[3];
};

template <typename T>
__global__ void k_cs_gather(SortArgs a) {
  const uint32_t cnt = cs_count(a);
  const T* d = static_cast<const T*>(a.d);
  const T* x = static_cast<const T*>(a.x);
  const T* n = static_cast<const T*>(a.n);
  SortRec<T>* out = reinterpret_cast<SortRec<T>*>(a.tmp);
  const size_t C = (size_t)a.cap;
  for (uint32_t k = blockIdx.x * blockDim.x + threadIdx.x; k < cnt; k += gridDim.x * blockDim.x) {
    const int32_t c = a.idx[k];
    SortRec<T> r;
    r.pi = a.pi[c]; r.pj = a.pj[c]; r.ti = a.ti[c]; r.tj = a.tj[c];
    r.d = d[c];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      r.x[q] = x[q * C + c];
      r.n[q] = n[q * C + c];
    }
    out[k] = r;
  }
}

template <typename T>
__global__ void k_cs_write(SortArgs a) {
  const uint32_t cnt = cs_count(a);
  T* d = static_cast<T*>(a.d);
  T* x = static_cast<T*>(a.x);
  T* n = static_cast<T*>(a.n);
  const SortRec<T>* in = reinterpret_cast<const SortRec<T>*>(a.tmp);
  const size_t C = (size_t)a.cap;
  for (uint32_t k = blockIdx.x * blockDim.x + threadIdx.x; k < cnt; k += gridDim.x * blockDim.x) {
    const SortRec<T> r = in[k];
    a.pi[k] = r.pi; a.pj[k] = r.pj; a.ti[k] = r.ti; a.tj[k] = r.tj;
    d[k] = r.d;
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      x[q * C + k] = r.x[q];
      n[q * C + k] = r.n[q];
    }
  }
}

// The adjoint rows move in a second pass through the same staging buffer
// (DEM_ADJOINT_ROWS values of the scene's precision per contact fit in a
// SortRec<double>).
static_assert(DEM_ADJOINT_ROWS * sizeof(double) <= sizeof(SortRec<double>), "adjoint rows exceed the staging record");

template <typename T>
__global__ void k_cs_gather_adj(SortArgs a) {
  const uint32_t cnt = cs_count(a);
  const T* adj = static_cast<const T*>(a.adj);
  T* out = reinterpret_cast<T*>(a.tmp);
  const size_t C = (size_t)a.cap;
  for (uint32_t k = blockIdx.x * blockDim.x + threadIdx.x; k < cnt; k += gridDim.x * blockDim.x) {
    const int32_t c = a.idx[k];
#pragma unroll
    for (int q = 0; q < DEM_ADJOINT_ROWS; ++q) out[(size_t)k * DEM_ADJOINT_ROWS + q] = adj[q * C + c];
  }
}

template <typename T>
__global__ void k_cs_write_adj(SortArgs a) {
  const uint32_t cnt = cs_count(a);
  T* adj = static_cast<T*>(a.adj);
  const T* in = reinterpret_cast<const T*>(a.tmp);
  const size_t C = (size_t)a.cap;
  for (uint32_t k = blockIdx.x * blockDim.x + threadIdx.x; k < cnt; k += gridDim.x * blockDim.x) {
#pragma unroll
    for (int q = 0; q < DEM_ADJOINT_ROWS; ++q) adj[q * C + k] = in[(size_t)k * DEM_ADJOINT_ROWS + q];
  }
}

SortLayout sort_layout(int32_t n_tris, int64_t cap) {
  SortLayout L;
  L.n_buckets = (uint32_t)n_tris + 1;
  L.n_blocks = (L.n_buckets + kSortChunk - 1) / kSortChunk;
  const size_t B = L.n_buckets, C = (size_t)std::max<int64_t>(cap, 1);
  size_t o = 0;
  L.hist = o; o = align_up(o + 4 * B, 256);
  L.fill = o; o = align_up(o + 4 * B, 256);
  L.bsum = o; o = align_up(o + 8 * ((size_t)L.n_blocks + 1), 256);
  L.idx = o; o = align_up(o + 4 * C, 256);
  L.tmp = o; o = align_up(o + sizeof(SortRec<double>) * C, 256);
  L.blist = o; o = align_up(o + 4 * (B + 1), 256);
  L.total = o;
  return L;
}

template <typename T>
dem_status run_sort(const dem_contacts* c, int32_t n_tris, void* ws, const SortLayout& L, uint32_t* status,
                    hipStream_t st) {
  char* base = static_cast<char*>(ws);
  SortArgs a;
  a.pi = c->pi; a.pj = c->pj; a.ti = c->ti; a.tj = c->tj;
  a.d = c->d; a.x = c->x; a.n = c->n;
  a.adj = c->adjoint;
  a.count = c->count;
  a.cap = c->capacity;
  a.n_buckets = L.n_buckets;
  a.hist = reinterpret_cast<uint32_t*>(base + L.hist);
  a.fill = reinterpret_cast<uint32_t*>(base + L.fill);
  a.bsum = reinterpret_cast<unsigned long long*>(base + L.bsum);
  a.idx = reinterpret_cast<int32_t*>(base + L.idx);
  a.tmp = base + L.tmp;
  a.blist = reinterpret_cast<uint32_t*>(base + L.blist);
  a.blist_n = a.blist + L.n_buckets;
  a.status = status;
  (void)n_tris;
  const dim3 g(2048), b(256);
  hipLaunchKernelGGL(k_cs_clear, dim3(4096), b, 0, st, a);
  hipLaunchKernelGGL(k_cs_count, g, b, 0, st, a);
  hipLaunchKernelGGL(k_cs_bsum, dim3(L.n_blocks), dim3(kSortThreads), 0, st, a);
  hipLaunchKernelGGL(k_cs_top, dim3(1), dim3(kScanThreads), 0, st, a, L.n_blocks);
  hipLaunchKernelGGL(k_cs_local, dim3(L.n_blocks), dim3(kSortThreads), 0, st, a);
  hipLaunchKernelGGL(k_cs_scatter, g, b, 0, st, a);
  hipLaunchKernelGGL(k_cs_list, dim3(4096), b, 0, st, a);
  hipLaunchKernelGGL(k_cs_small, g, b, 0, st, a);
  hipLaunchKernelGGL(k_cs_bucket, dim3(4096), b, 0, st, a);
  hipLaunchKernelGGL(k_cs_gather<T>, g, b, 0, st, a);
  hipLaunchKernelGGL(k_cs_write<T>, g, b, 0, st, a);
  if (a.adj) {
    hipLaunchKernelGGL(k_cs_gather_adj<T>, g, b, 0, st, a);
    hipLaunchKernelGGL(k_cs_write_adj<T>, g, b, 0, st, a);
  }
  return hipGetLastError() == hipSuccess ? DEM_OK : DEM_ERR_HIP;
}

}  // namespace

// Device scratch of dem_find_contacts_noalloc: the workspace (soup, level
// queues, near list, counters) of callers that cannot allocate device memory.
// One copy per GPU, held until the process ends.  In host code `scratch`
// names a host-side stand-in, never the device memory itself: its device
// address is looked up once per device (hipGetSymbolAddress, with that
// device current) and only that address is passed to kernels.
static __device__ __align__(256) uint8_t scratch[DEM_SCRATCH_BYTES];

namespace {

constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_addr[kMaxScratchDevices] = {};

// Device address of `scratch` on the current device (looked up on the
// first call on that device).
dem_status scratch_address(void** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxScratchDevices) return DEM_ERR_HIP;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_addr[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return DEM_ERR_HIP;
    if (reinterpret_cast<uintptr_t>(ptr) % 256) return DEM_ERR_HIP;
    g_scratch_addr[dev] = ptr;
  }
  *out = g_scratch_addr[dev];
  return DEM_OK;
}

// Argument checks shared by dem_find_contacts and its no-allocation variant.
dem_status find_args_ok(const dem_scene* scene, const int32_t* pairs, int32_t n_pairs, const dem_params& p,
                        const dem_contacts* out, const uint32_t* dev_status) {
  if (!scene_ok(scene) || !params_ok(p)) return DEM_ERR_ARG;
  if (n_pairs < 0 || (n_pairs > 0 && !pairs)) return DEM_ERR_ARG;
  if (!out || !out->count || out->capacity < 0 || out->capacity > (int64_t)0xFFFFFFFF) return DEM_ERR_ARG;
  if (out->capacity > 0 && (!out->pi || !out->pj || !out->ti || !out->tj || !out->d || !out->x || !out->n))
    return DEM_ERR_ARG;
  if (!dev_status) return DEM_ERR_ARG;
  return DEM_OK;
}

dem_status find_dispatch(const dem_scene* scene, const int32_t* pairs, int32_t n_pairs, const dem_params& p,
                         const dem_contacts* out, void* ws, const WsLayout& L, dem_stats* dev_stats,
                         uint32_t* dev_status, double* dev_energy, hipStream_t st) {
  if (scene->precision == DEM_F64)
    return run_find<double>(scene, pairs, n_pairs, p, out, ws, L, dev_stats, dev_status, dev_energy, st);
  return run_find<float>(scene, pairs, n_pairs, p, out, ws, L, dev_stats, dev_status, dev_energy, st);
}

template <typename T>
void launch_backward(int grid, hipStream_t st, const SoupRec<T>* soup, const dem_scene* scene, const dem_contacts* c,
                     double k, const double* grad_E, T* grad, double* energy, uint32_t* status) {
  const T* cd = static_cast<const T*>(c->d);
  const T* adj = static_cast<const T*>(c->adjoint);
  const auto a16 = [](const void* q) { return reinterpret_cast<uintptr_t>(q) % 16 == 0; };
  const bool vec = c->capacity % 4 == 0 && a16(c->ti) && a16(c->tj) && a16(cd) && a16(adj);
  if (adj && cd && vec)
    hipLaunchKernelGGL((k_backward<T, true, true>), dim3(grid), dim3(256), 0, st, soup, scene->tri_verts,
                       scene->n_tris, scene->n_verts, c->ti, c->tj, cd, adj, c->count, c->capacity, k, grad_E, grad,
                       energy, status);
  else if (adj && cd)
    hipLaunchKernelGGL((k_backward<T, true, false>), dim3(grid), dim3(256), 0, st, soup, scene->tri_verts,
                       scene->n_tris, scene->n_verts, c->ti, c->tj, cd, adj, c->count, c->capacity, k, grad_E, grad,
                       energy, status);
  else
    hipLaunchKernelGGL((k_backward<T, false, false>), dim3(grid), dim3(256), 0, st, soup, scene->tri_verts,
                       scene->n_tris, scene->n_verts, c->ti, c->tj, cd, adj, c->count, c->capacity, k, grad_E, grad,
                       energy, status);
}

}  // namespace

extern "C" {

void dem_default_params(dem_params* p) {
  if (!p) return;
  std::memset(p, 0, sizeof(*p));
  p->mode = DEM_MODE_HIER;
  p->n_iter = 4;
  p->omega = 1.0f;
  p->alpha_reg_rel = 1e-4f;
  p->alpha_it_ratio = 1e3f;
  p->init_centroid = 0;
  p->dense_distance = 0;
  p->certify = 0;
  p->energy_k = 1e4;
  p->block = 256;
  p->grid = 1024;
  p->batch_items = 128;
  p->flat_tile_i = 256;
  p->flat_tile_j = 64;
  p->seed_chunk = 8;
  p->queue_capacity = 1 << 22;
  p->near_capacity = 1 << 22;
}

size_t dem_workspace_bytes(const dem_scene* scene, int32_t n_pairs, const dem_params* pp) {
  dem_params p;
  if (pp) p = *pp; else dem_default_params(&p);
  if (!scene_ok(scene) || !params_ok(p) || n_pairs < 0) return 0;
  return ws_layout(scene->precision, scene->n_tris, p.queue_capacity, p.near_capacity).total;
}

dem_status dem_find_contacts(const dem_scene* scene, const int32_t* pairs, int32_t n_pairs,
                             const dem_params* pp, const dem_contacts* out, void* workspace,
                             size_t workspace_bytes, dem_stats* dev_stats, uint32_t* dev_status,
                             double* dev_energy, dem_stream_t stream) {
  dem_params p;
  if (pp) p = *pp; else dem_default_params(&p);
  const dem_status a = find_args_ok(scene, pairs, n_pairs, p, out, dev_status);
  if (a != DEM_OK) return a;
  if (!workspace) return DEM_ERR_ARG;
  WsLayout L = ws_layout(scene->precision, scene->n_tris, p.queue_capacity, p.near_capacity);
  if (workspace_bytes < L.total) return DEM_ERR_CAPACITY;
  if (reinterpret_cast<uintptr_t>(workspace) % 256) return DEM_ERR_ARG;
  return find_dispatch(scene, pairs, n_pairs, p, out, workspace, L, dev_stats, dev_status, dev_energy,
                       reinterpret_cast<hipStream_t>(stream));
}

dem_status dem_find_contacts_noalloc(const dem_scene* scene, const int32_t* pairs, int32_t n_pairs,
                                     const dem_params* pp, const dem_contacts* out, dem_stats* dev_stats,
                                     uint32_t* dev_status, double* dev_energy, dem_stream_t stream) {
  dem_params p;
  if (pp) p = *pp; else dem_default_params(&p);
  const dem_status a = find_args_ok(scene, pairs, n_pairs, p, out, dev_status);
  if (a != DEM_OK) return a;
  WsLayout L = ws_layout(scene->precision, scene->n_tris, p.queue_capacity, p.near_capacity);
  if (L.total > (size_t)DEM_SCRATCH_BYTES) return DEM_ERR_CAPACITY;
  void* ws = nullptr;
  const dem_status sa = scratch_address(&ws);
  if (sa != DEM_OK) return sa;
  return find_dispatch(scene, pairs, n_pairs, p, out, ws, L, dev_stats, dev_status, dev_energy,
                       reinterpret_cast<hipStream_t>(stream));
}

dem_status dem_contact_backward(const dem_scene* scene, const dem_contacts* c, double k,
                                const double* grad_E, void* grad_verts, double* energy_out,
                                const void* workspace, size_t workspace_bytes, uint32_t* dev_status,
                                dem_stream_t stream) {
  if (!scene_ok(scene) || !c || !c->count || !c->ti || !c->tj || !dev_status) return DEM_ERR_ARG;
  if (!grad_verts && !energy_out) return DEM_ERR_ARG;
  if (!(k >= 0.0)) return DEM_ERR_ARG;
  if (c->capacity < 0 || c->capacity > (int64_t)0xFFFFFFFF) return DEM_ERR_ARG;
  // with adjoint rows nothing is read from the workspace
  const bool rows = c->adjoint && c->d;
  WsLayout L = ws_layout(scene->precision, scene->n_tris, 1, 1);
  if (!rows) {
    if (!workspace) return DEM_ERR_ARG;
    if (workspace_bytes < L.qa) return DEM_ERR_CAPACITY;
    if (reinterpret_cast<uintptr_t>(workspace) % 256) return DEM_ERR_ARG;
  }
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  const char* base = rows ? nullptr : static_cast<const char*>(workspace);
  if (energy_out) hipLaunchKernelGGL(k_zero_scalar, dim3(1), dim3(64), 0, st, energy_out);
  const int grid = 1024;
  if (scene->precision == DEM_F64)
    launch_backward<double>(grid, st, rows ? nullptr : reinterpret_cast<const SoupRec<double>*>(base + L.soup), scene, c, k, grad_E,
                            static_cast<double*>(grad_verts), energy_out, dev_status);
  else
    launch_backward<float>(grid, st, rows ? nullptr : reinterpret_cast<const SoupRec<float>*>(base + L.soup), scene, c, k, grad_E,
                           static_cast<float*>(grad_verts), energy_out, dev_status);
  return hipGetLastError() == hipSuccess ? DEM_OK : DEM_ERR_HIP;
}

size_t dem_frontier_workspace_bytes(const dem_scene* scene, int32_t n_pairs, const dem_params* pp,
                                    int64_t frontier_capacity) {
  dem_params p;
  if (pp) p = *pp; else dem_default_params(&p);
  if (!scene_ok(scene) || !params_ok(p) || n_pairs < 0) return 0;
  if (frontier_capacity < 1 || frontier_capacity > (int64_t)0xFFFFFFFF) return 0;
  return fr_layout(scene->precision, scene->n_tris, p.near_capacity, frontier_capacity, fr_grid(p), n_pairs)
      .total;
}

dem_status dem_frontier_init(const dem_scene* scene, const int32_t* pairs, int32_t n_pairs,
                             const dem_params* pp, const dem_frontier* f, void* workspace,
                             size_t workspace_bytes, uint32_t* dev_status, dem_stream_t stream) {
  dem_params p;
  if (pp) p = *pp; else dem_default_params(&p);
  if (!scene_ok(scene) || !params_ok(p) || !frontier_ok(f) || !dev_status || !workspace) return DEM_ERR_ARG;
  if (n_pairs < 0 || (n_pairs > 0 && !pairs)) return DEM_ERR_ARG;
  if (reinterpret_cast<uintptr_t>(workspace) % 256) return DEM_ERR_ARG;
  FrLayout FL = fr_layout(scene->precision, scene->n_tris, p.near_capacity, f->capacity, fr_grid(p), n_pairs);
  if (workspace_bytes < FL.total) return DEM_ERR_CAPACITY;
  unsigned long long* pc = reinterpret_cast<unsigned long long*>(static_cast<char*>(workspace) + FL.pcount);
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  hipLaunchKernelGGL(k_fr_mem_clear, dim3(1024), dim3(256), 0, st,
                     reinterpret_cast<unsigned long long*>(f->memory), f->memory_capacity);
  if (n_pairs > 0)
    hipLaunchKernelGGL(k_fr_init_count, dim3((n_pairs + 255) / 256), dim3(256), 0, st, pairs, n_pairs,
                       scene->root_count, pc);
  hipLaunchKernelGGL(k_fr_init_scan, dim3(1), dim3(kScanThreads), 0, st, pc, n_pairs, f->state, f->capacity,
                     dev_status);
  if (n_pairs > 0)
    hipLaunchKernelGGL(k_fr_init_write, dim3(std::min(n_pairs, 65535)), dim3(256), 0, st, pairs, n_pairs,
                       scene->root_begin, scene->root_count, pc, f->capacity,
                       reinterpret_cast<int4*>(f->leaves[0]));
  return hipGetLastError() == hipSuccess ? DEM_OK : DEM_ERR_HIP;
}

dem_status dem_frontier_step(const dem_scene* scene, const dem_params* pp, const dem_frontier* f,
                             const dem_contacts* out, void* workspace, size_t workspace_bytes,
                             dem_stats* dev_stats, uint32_t* dev_status, double* dev_energy,
                             dem_stream_t stream) {
  dem_params p;
  if (pp) p = *pp; else dem_default_params(&p);
  if (!scene_ok(scene) || !params_ok(p) || !frontier_ok(f)) return DEM_ERR_ARG;
  if (!scene->tri_parent || !scene->tri_depth) return DEM_ERR_ARG;
  if (!out || !out->count || out->capacity < 0 || out->capacity > (int64_t)0xFFFFFFFF) return DEM_ERR_ARG;
  if (out->capacity > 0 && (!out->pi || !out->pj || !out->ti || !out->tj || !out->d || !out->x || !out->n))
    return DEM_ERR_ARG;
  if (!workspace || !dev_status) return DEM_ERR_ARG;
  FrLayout FL = fr_layout(scene->precision, scene->n_tris, p.near_capacity, f->capacity, fr_grid(p), 0);
  if (workspace_bytes < FL.total) return DEM_ERR_CAPACITY;
  if (reinterpret_cast<uintptr_t>(workspace) % 256) return DEM_ERR_ARG;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  if (scene->precision == DEM_F64)
    return run_frontier_step<double>(scene, p, f, out, workspace, FL, dev_stats, dev_status, dev_energy, st);
  return run_frontier_step<float>(scene, p, f, out, workspace, FL, dev_stats, dev_status, dev_energy, st);
}

size_t dem_sort_contacts_workspace_bytes(const dem_scene* scene, int64_t contact_capacity) {
  if (!scene || scene->n_tris <= 0 || contact_capacity < 0 || contact_capacity > (int64_t)0xFFFFFFFF) return 0;
  return sort_layout(scene->n_tris, contact_capacity).total;
}

dem_status dem_sort_contacts(const dem_scene* scene, const dem_contacts* c, void* workspace, size_t workspace_bytes,
                             uint32_t* dev_status, dem_stream_t stream) {
  if (!scene_ok(scene) || !c || !c->count || !dev_status || !workspace) return DEM_ERR_ARG;
  if (c->capacity < 0 || c->capacity > (int64_t)0xFFFFFFFF) return DEM_ERR_ARG;
  if (c->capacity > 0 && (!c->pi || !c->pj || !c->ti || !c->tj || !c->d || !c->x || !c->n)) return DEM_ERR_ARG;
  const SortLayout L = sort_layout(scene->n_tris, c->capacity);
  if (workspace_bytes < L.total) return DEM_ERR_CAPACITY;
  if (reinterpret_cast<uintptr_t>(workspace) % 256) return DEM_ERR_ARG;
  if (c->capacity == 0) return DEM_OK;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  if (scene->precision == DEM_F64) return run_sort<double>(c, scene->n_tris, workspace, L, dev_status, st);
  return run_sort<float>(c, scene->n_tris, workspace, L, dev_status, st);
}

size_t dem_contact_forces_workspace_bytes(int64_t contact_capacity) {
  if (contact_capacity < 0 || contact_capacity > (int64_t)0x7FFFFFFF) return 0;
  return cf_layout(std::max<int64_t>(contact_capacity, 1)).total;
}

dem_status dem_contact_forces(const dem_scene* scene, const dem_contacts* c, const void* mass,
                              const void* centre, double k_s, double merge_scale, const dem_merged* out,
                              int32_t* group, void* force, void* torque, void* workspace,
                              size_t workspace_bytes, uint32_t* dev_status, dem_stream_t stream) {
  if (!scene_ok(scene) || !c || !c->count || !out || !out->count || !mass || !centre || !dev_status || !workspace)
    return DEM_ERR_ARG;
  if (c->capacity < 0 || c->capacity > (int64_t)0x7FFFFFFF) return DEM_ERR_ARG;
  if (c->capacity > 0 && (!c->pi || !c->pj || !c->ti || !c->tj || !c->x || !c->n)) return DEM_ERR_ARG;
  if (out->capacity < 0 || out->capacity > (int64_t)0xFFFFFFFF) return DEM_ERR_ARG;
  if (out->capacity > 0 && (!out->pi || !out->pj || !out->x || !out->n || !out->f || !out->members))
    return DEM_ERR_ARG;
  if (!(k_s >= 0.0) || !(k_s < INFINITY) || !(merge_scale >= 0.0) || !(merge_scale < INFINITY)) return DEM_ERR_ARG;
  if (reinterpret_cast<uintptr_t>(workspace) % 256) return DEM_ERR_ARG;
  CfLayout L = cf_layout(std::max<int64_t>(c->capacity, 1));
  if (workspace_bytes < L.total) return DEM_ERR_CAPACITY;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  if (scene->precision == DEM_F64)
    return run_forces<double>(scene, c, mass, centre, k_s, merge_scale, out, group, force, torque, workspace, L,
                              dev_status, st);
  return run_forces<float>(scene, c, mass, centre, k_s, merge_scale, out, group, force, torque, workspace, L,
                           dev_status, st);
}

const char* dem_status_string(dem_status s) {
  switch (s) {
    case DEM_OK: return "ok";
    case DEM_ERR_ARG: return "invalid argument";
    case DEM_ERR_CAPACITY: return "workspace too small";
    case DEM_ERR_HIP: return "HIP error";
    case DEM_ERR_NOT_CONSERVATIVE: return "hierarchy violates the surrogate-tree rules";
    case DEM_ERR_OOM: return "host allocation failed";
  }
  return "unknown status";
}

const char* dem_version(void) { return "dem 0.1 gfx950"; }

}  // extern "C"
