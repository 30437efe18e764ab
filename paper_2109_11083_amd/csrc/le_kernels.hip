// le_kernels.hip -- gfx950 kernels of the Lees-Edwards shear-flow MD step.
//
// Compiled with -ffp-contract=off: every product and sum below rounds as
// written, which keeps the boundary crossing, cell index and pair
// displacement bit-identical to their plain definitions; fused multiply-adds
// are requested explicitly (fma) only where results are compared with a
// tolerance (force law, accumulations).
//
// Data layout (all cell-sorted by (cell id, tag), re-sorted at every
// neighbour-list build):
//   positions  double4 AoS (x, y, z, unused) -- one 32-byte gather per neighbour
//   velocities, forces  float64 SoA [3][np] -- streamed, coalesced
//   neighbour list  int32 [K][np] (row-major by neighbour index, so that the
//                   k-th entries of 64 consecutive particles are contiguous)
#include <math.h>

#include <hip/hip_ext.h>

#include "le_internal.h"

namespace le {

// ---------------------------------------------------------------- helpers
__device__ __forceinline__ int xcd_map(int b, int nblocks) {
  // Blocks are dealt round-robin to the 8 XCDs; remap so that each XCD works
  // on one contiguous range of cell-sorted particles (its L2 then holds that
  // region's neighbour positions).
  const int X = 8;
  int q = nblocks / X, r = nblocks % X;
  int x = b % X, k = b / X;
  return x * q + (x < r ? x : r) + k;
}
__device__ __forceinline__ int xcd_block(int nblocks) { return xcd_map((int)blockIdx.x, nblocks); }

// The other way round: runs of C consecutive blocks are dealt round-robin to
// the XCDs, so that any stretch of the grid (the tiles of the members of a
// batch that rebuild at this step) is spread over all of them.
template <int C>
__device__ __forceinline__ int xcd_spread(int b, int nblocks) {
  const int X = 8, G = X * C;
  const int full = nblocks / G * G;
  if (b >= full) return b;
  const int x = b % X, k = b / X;
  return ((k / C) * X + x) * C + k % C;
}

// Simulation and local block of global block g of a batched launch: the last
// simulation whose first block is at or before g (simulations without blocks
// are skipped).  Uniform across the block.
__device__ __forceinline__ void locate(const Batch& b, int g, int& sim, int& bid) {
  int lo = 0, hi = b.nsims - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (b.start[mid] <= g) lo = mid; else hi = mid - 1;
  }
  sim = lo;
  bid = g - b.start[lo];
}

// The descriptor of a batched launch's simulation.  It never changes while
// kernels run (written once at le_init), so it is read as constant memory:
// through an address-space-4 pointer the loads become scalar loads into SGPRs,
// as for the by-value descriptor of a single-simulation launch.
static_assert(sizeof(Dev) % 8 == 0, "the descriptor is a whole number of 8-byte words");
typedef const __attribute__((address_space(4))) Dev ConstDev;
__device__ __forceinline__ const Dev& stage_dev(const Dev* src) {
  return *(const Dev*)(ConstDev*)src;
}

__device__ __forceinline__ void latch(Flags* f, int32_t st) { atomicCAS(&f->status, 0, st); }

// Canonical periodic wrap into [0, L); returns the net number of box lengths
// subtracted (the Lees-Edwards crossing count for the gradient axis).
__device__ __forceinline__ double wrap1(double& x, double L) {
  double k = floor(x / L);
  double v = x - k * L;
  if (v < 0.0) { v += L; k -= 1.0; }
  if (v >= L) { v -= L; k += 1.0; }
  x = v;
  return k;
}

// The fourth word of each position holds the particle's wrap counts along y
// and z since le_init (two int32 in the bits of the double; only ever copied,
// never used in arithmetic).
__device__ __forceinline__ void img_get(double w, int& ky, int& kz) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(w);
  ky = (int)(uint32_t)(b >> 32);
  kz = (int)(uint32_t)(b & 0xffffffffull);
}
__device__ __forceinline__ double img_put(int ky, int kz) {
  const unsigned long long b = ((unsigned long long)(uint32_t)ky << 32) | (unsigned long long)(uint32_t)kz;
  return __longlong_as_double((long long)b);
}


__device__ __forceinline__ int cell_index(double v, double inv, int n) {
  int k = (int)(v * inv);
  if (k < 0) k = 0;
  if (k > n - 1) k = n - 1;
  return k;
}

__device__ __forceinline__ int floor_div(int a, int b) {
  int q = a / b;
  if ((a % b != 0) && ((a < 0) != (b < 0))) --q;
  return q;
}

__device__ __forceinline__ double wave_max(double v) {
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

// Philox4x32-10: two 32x32->64 products per round with the published
// multipliers, key advanced by the published Weyl increments between rounds.
__device__ __forceinline__ void philox(uint32_t c[4], uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r > 0) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
    // one 32 x 32 -> 64-bit product per multiplier (a single v_mad_u64_u32)
    const uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c[0];
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c[2];
    uint32_t lo0 = (uint32_t)p0, hi0 = (uint32_t)(p0 >> 32);
    uint32_t lo1 = (uint32_t)p1, hi1 = (uint32_t)(p1 >> 32);
    uint32_t n0 = hi1 ^ c[1] ^ k0;
    uint32_t n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0; c[1] = lo1; c[2] = n2; c[3] = lo0;
  }
}

__device__ __forceinline__ double u01c(uint32_t r) {
  return ((double)r + 0.5) * (1.0 / 4294967296.0) - 0.5;
}

// ---------------------------------------------------------- state loading
__global__ void k_load_state(Dev d, const double* __restrict__ x0, const double* __restrict__ u0,
                             const double* __restrict__ f0, int64_t step0, double Delta0) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int n = d.n, np = d.np;
  if (i < n) {
    double4 p;
    p.x = x0[i]; p.y = x0[n + i]; p.z = x0[2 * n + i]; p.w = 0.0;
    reinterpret_cast<double4*>(d.pos[0])[i] = p;
    for (int a = 0; a < 3; ++a) {
      d.vel[0][a * np + i] = u0 ? u0[a * n + i] : 0.0;  // no velocities: particles at rest
      d.frc[0][a * np + i] = f0 ? f0[a * n + i] : 0.0;
    }
    d.tag[0][i] = i;
  }
  if (i == 0) {
    // far-away sentinel at slot n pads neighbour batches: r^2 ~ 1e200 never passes a cutoff
    const double4 far = make_double4(1e100, 1e100, 1e100, 0.0);
    reinterpret_cast<double4*>(d.pos[0])[n] = far;
    reinterpret_cast<double4*>(d.pos[1])[n] = far;
  }
  for (int c = i; c < d.ncell; c += gridDim.x * blockDim.x) d.cell_count[c] = 0;
  if (i == 0) {
    Ctrl* c = d.ctrl;
    c->step = step0;
    c->rebuild_step = step0;
    c->n_rebuilds = 0;
    c->Delta = Delta0;
    c->Delta_ref = Delta0;
    c->drift = 0.0;
    c->pos_cur = 0;
    c->aux_cur = 0;
    c->rebuild = 0;
    c->wraps = 0;
    d.flags->status = 0;
    for (int k = 0; k < kSlots * kLineInts; ++k) d.flags->max_nb_slot[k] = 0;
  }
  for (int k = i; k < kSlots * kLineU64; k += gridDim.x * blockDim.x) d.vmax[k] = 0ull;
}

// ------------------------------------------------------------- rebuild
// Three kernels, each an empty launch unless the lists are rebuilt for the
// current state: (1) advance the step and decide, then crossing + wrap + bin,
// (2) cell-count scan and, block by block, rank by tag + permute, (3)
// neighbour lists.

// Advance the step counter and the offset, adopt the drifted positions, and
// decide whether the neighbour lists must be rebuilt before the next force
// evaluation.  Pair displacements evolve as d' = d + dt (c_i - c_j) +
// gamma_dot dt d_y e_x, so after a strain s = |gamma_dot| (t - t_build) and a
// peculiar path bound D = sum dt max|c|, a pair within rc now was within
// g (rc + 2 g D) at the build, g = s/2 + sqrt(1 + s^2/4) the norm of the
// inverse shear.  The lists (radius rc + skin) stay complete while that bound
// is below rc + skin.  Pure: every block evaluates it on its own copy.
__device__ __forceinline__ void control_advance(const Dev& d, Ctrl& c, unsigned long long vbits) {
  double vmax = sqrt(__longlong_as_double((long long)vbits));
  c.drift += d.dt * vmax;
  c.step += 1;
  c.Delta = le_offset(c.step, d.dt, d.sv, d.Lx);
  c.pos_cur ^= 1;
  double T = (double)(c.step - c.rebuild_step) * d.dt;
  c.wraps = (int)rint((c.Delta_ref + d.sv * T - c.Delta) / d.Lx);
  double s = fabs(d.shear_rate) * T;
  double g = 0.5 * s + sqrt(1.0 + 0.25 * s * s);
  double rc = sqrt(d.rc2);
  double need = g * (rc + 2.0 * g * c.drift);
  c.rebuild = (d.rlist <= rc || need >= d.rlist * (1.0 - 1e-9)) ? 1 : 0;
}

// The bookkeeping of a rebuild, applied to the state the rebuild produces:
// sorted copies go to the other buffers, the offset and step become the
// reference of the co-moving criterion.
__device__ __forceinline__ void rebuild_adopt(Ctrl& c) {
  c.pos_cur ^= 1;
  c.aux_cur ^= 1;
  c.rebuild = 1;
  c.rebuild_step = c.step;
  c.Delta_ref = c.Delta;
  c.drift = 0.0;
  c.wraps = 0;
  c.n_rebuilds += 1;
}

// (both words read unconditionally, so that the two loads overlap: this is
// all an empty launch of the chain does)
__device__ __forceinline__ bool rebuild_off(const Dev& d) {
  const int status = d.flags->status;
  const int rebuild = d.ctrl->rebuild;
  return (status != 0) | (rebuild == 0);
}

// (1) Reads control copy d.ctrl and writes the next one (block 0).  With
// `control` the step is advanced first (after a drift).  On a rebuild:
// boundary crossing (Lees-Edwards shift and velocity jump) + periodic wrap of
// x and z in place, then each particle's tag and slot go into its cell's bucket at
// its arrival rank.  Runs of equal cells within a wave take one atomic per run.
__device__ __forceinline__ void control_bin_body(const Dev& d, Ctrl* __restrict__ next,
                                                 unsigned long long* __restrict__ next_vmax, int force,
                                                 int control, int bid) {
  __shared__ Ctrl sc;
  __shared__ int go;
  if (threadIdx.x < 64) {
    // the drift's speed bound: max over the slot words (first wave)
    unsigned long long vb = threadIdx.x < kSlots ? d.vmax[threadIdx.x * kLineU64] : 0ull;
    for (int o = 32; o > 0; o >>= 1) {
      unsigned long long t = __shfl_xor(vb, o, 64);
      vb = t > vb ? t : vb;
    }
    const bool ok = d.flags->status == 0;
    Ctrl c = *d.ctrl;
    if (ok && control) control_advance(d, c, vb);
    const bool rb = ok && (force || c.rebuild);
    if (threadIdx.x == 0) {
      sc = c;  // buffers and offset of the state being binned
      go = rb ? 1 : 0;
    }
    if (bid == 0) {
      if (threadIdx.x < kSlots) next_vmax[threadIdx.x * kLineU64] = 0ull;
      if (rb)
        for (int k = threadIdx.x; k < kSlots * kLineInts; k += 64) d.flags->max_nb_slot[k] = 0;
      if (threadIdx.x == 0) {
        Ctrl o = c;
        o.rebuild = 0;
        if (rb) rebuild_adopt(o);
        *next = o;
      }
    }
  }
  __syncthreads();
  if (!go) return;
  // the look-back words of the scan start cleared (spread over the blocks)
  const int nbb = (d.n + kBinBlock - 1) / kBinBlock;  // blocks of this pass
  for (int k = bid * kBlock + (int)threadIdx.x; k < d.sp_blocks; k += nbb * kBlock) d.scan_status[k] = 0ull;
  const int np = d.np;
  for (int rd = 0; rd < kBinBlock / kBlock; ++rd) {
    const int i = bid * kBinBlock + rd * kBlock + (int)threadIdx.x;
    int cell = -1, tg = 0;
    if (i < d.n) {
      tg = d.tag[sc.aux_cur][i];
      double4* P = reinterpret_cast<double4*>(d.pos[sc.pos_cur]);
      double* U = d.vel[sc.aux_cur];
      double4 p = P[i];
      double x = p.x, y = p.y, z = p.z;
      double ux = U[i];
      const double Delta = sc.Delta;
      double ky = wrap1(y, d.Ly);
      x = x - ky * Delta;
      ux = ux - ky * d.jump_sv;  // velocity jump (lab storage only)
      wrap1(x, d.Lx);
      double kz = wrap1(z, d.Lz);
      int cy, cz;
      img_get(p.w, cy, cz);
      p.w = img_put(cy + (int)ky, cz + (int)kz);
      double uy = U[np + i], uz = U[2 * np + i];
      if (!(isfinite(x) && isfinite(y) && isfinite(z) && isfinite(ux) && isfinite(uy) && isfinite(uz))) {
        latch(d.flags, LE_E_NONFINITE);
        x = 0.0; y = 0.0; z = 0.0;
      }
      p.x = x; p.y = y; p.z = z;
      P[i] = p;
      U[i] = ux;
      int ix = cell_index(x, d.inv_lx, d.nx);
      int iy = cell_index(y, d.inv_ly, d.ny);
      int iz = cell_index(z, d.inv_lz, d.nz);
      cell = (iz * d.ny + iy) * d.nx + ix;
    }
    // runs of equal cells among consecutive lanes share one atomic
    const int lane = threadIdx.x & 63;
    const int prev = __shfl_up(cell, 1, 64);
    const bool head = lane == 0 || prev != cell;
    const unsigned long long heads = __ballot(head);
    const int run0 = 63 - __clzll(heads & ((2ull << lane) - 1ull));  // lane 63: mask all ones
    const unsigned long long after = lane == 63 ? 0ull : (heads & ~((2ull << lane) - 1ull));
    const int run1 = after ? __ffsll((long long)after) - 1 : 64;  // first lane of the next run
    int base = 0;
    if (head && cell >= 0) base = atomicAdd(&d.cell_count[cell], run1 - lane);
    base = __shfl(base, run0, 64);
    if (cell >= 0) {
      const int r = base + (lane - run0);
      if (r < d.bcap) d.bucket[(size_t)cell * d.bcap + r] = make_int2(tg, i);
      else latch(d.flags, LE_E_CAPACITY);
    }
  }
}

__global__ void __launch_bounds__(kBlock) k_control_bin(Dev d, Ctrl* __restrict__ next,
                                                        unsigned long long* __restrict__ next_vmax,
                                                        int force, int control) {
  control_bin_body(d, next, next_vmax, force, control, blockIdx.x);
}

// Batched form: every simulation advances its step (control) and writes its
// other control copy (named by its descriptor).
__global__ void __launch_bounds__(kBlock) k_control_bin_b(Batch b) {
  int sm, bid;
  locate(b, blockIdx.x, sm, bid);
  const Dev& d = stage_dev(b.dev[sm]);
  control_bin_body(d, d.ctrl_other, d.vmax_other, 0, 1, bid);
}

// (2) One pass over the cells in blocks of sp_cells consecutive cells.  The
// exclusive scan of the cell counts into cell_start uses decoupled
// look-back: block b publishes its total in status word b (flag 1), adds the
// totals of its predecessors walking back (64 at a time, one per lane of the
// first wave) until one has published its inclusive prefix (flag 2), and
// publishes its own.  A word packs flag << 62 | value, so one 64-bit atomic
// carries both.  Every block publishes its total before it waits, and blocks
// start in grid order, so the oldest unfinished block never waits on one
// that has not started: every wait ends; a bounded spin latches LE_E_STATE
// rather than hang.  The counts are cleared for the next binning pass.
//
// With its slots known, the block moves the particles of its own cells: the
// final slot of a particle is its cell's start plus the number of cell-mates
// with a smaller tag, so the order is (cell, tag) whatever the arrival order.
// The bucket entry carries the particle's binned slot; its state is copied
// from there to the final slot in the other buffers.  No block reads what
// another writes, so the sort needs no further pass.
__device__ __forceinline__ unsigned long long scan_word(int flag, long long v) {
  return ((unsigned long long)flag << 62) | (unsigned long long)v;
}

__device__ __forceinline__ void scan_permute_body(const Dev& d, int b) {
  if (rebuild_off(d)) return;
  __shared__ int lpre[kBlock + 1];  // exclusive prefix of the block's counts, total last
  __shared__ int wsum[kBlock / 64];
  __shared__ long long base_sh;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int c0 = b * d.sp_cells;
  const int ncb = min(d.sp_cells, d.ncell - c0);  // cells of this block (>= 1)
  const int v = (int)threadIdx.x < ncb ? d.cell_count[c0 + threadIdx.x] : 0;
  int incl = v;
  for (int o = 1; o < 64; o <<= 1) {
    int t = __shfl_up(incl, o, 64);
    if (lane >= o) incl += t;
  }
  if (lane == 63) wsum[wid] = incl;
  __syncthreads();
  int woff = 0, agg = 0;
  for (int w = 0; w < kBlock / 64; ++w) {
    if (w < wid) woff += wsum[w];
    agg += wsum[w];
  }
  if ((int)threadIdx.x < ncb) lpre[threadIdx.x] = woff + incl - v;
  if (threadIdx.x == 0) lpre[ncb] = agg;
  if (wid == 0) {
    // look back with the whole first wave: lane l reads the word of block
    // p - l, so one round covers 64 predecessors; the prefix is the sum of
    // the aggregates up to and including the nearest inclusive prefix
    unsigned long long* st = d.scan_status;
    const unsigned long long vmask = (1ull << 62) - 1ull;
    long long prefix = 0;
    if (lane == 0)
      __hip_atomic_store(&st[b], scan_word(b == 0 ? 2 : 1, agg), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    int p = b - 1;
    long long spins = 0;
    while (p >= 0) {
      const int q = p - lane;
      // before block 0 the prefix is an inclusive 0
      const unsigned long long w =
          q >= 0 ? __hip_atomic_load(&st[q], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : scan_word(2, 0);
      const int flag = (int)(w >> 62);
      const unsigned long long inc = __ballot(flag == 2);
      const unsigned long long zero = __ballot(flag == 0);
      const int first2 = inc ? __builtin_ctzll(inc) : 64;
      const unsigned long long need = first2 >= 63 ? ~0ull : ((2ull << first2) - 1ull);
      if (zero & need) {  // a predecessor in reach has not published yet
        if (++spins > (1ll << 22)) {
          if (lane == 0) latch(d.flags, LE_E_STATE);
          prefix = -1;  // no prefix: the block moves nothing
          break;
        }
        __builtin_amdgcn_s_sleep(1);
        continue;
      }
      long long val = lane <= first2 ? (long long)(w & vmask) : 0;
      for (int o = 32; o > 0; o >>= 1) val += __shfl_xor(val, o, 64);
      prefix += val;
      if (first2 < 64) break;
      p -= 64;
    }
    if (lane == 0) {
      if (b > 0 && prefix >= 0)
        __hip_atomic_store(&st[b], scan_word(2, prefix + agg), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      base_sh = prefix;
    }
  }
  __syncthreads();
  if (base_sh < 0) return;
  const int base = (int)base_sh;
  if ((int)threadIdx.x < ncb) {
    d.cell_start[c0 + threadIdx.x] = base + lpre[threadIdx.x];
    d.cell_count[c0 + threadIdx.x] = 0;
  }
  if (c0 + ncb == d.ncell && threadIdx.x == 0) d.cell_start[d.ncell] = base + agg;  // = n

  // the block's particles, two per thread and round (their loads overlap):
  // k-th cell of the block with lpre[k] <= f < lpre[k + 1], arrival rank
  // r = f - lpre[k]; the bucket entry holds the tag and the binned slot
  const Ctrl* c = d.ctrl;
  const int np = d.np;
  const int pd = c->pos_cur, ad = c->aux_cur;  // destination buffers
  const int ps = 1 - pd, as = 1 - ad;          // binned (source) buffers
  // the final slot (-1: none), binned slot and tag of the block's f-th particle
  auto locate_f = [&](int f, int& ns, int& src, int& tg) {
    ns = -1;
    src = 0;
    tg = 0;
    if (f >= agg) return;
    int lo = 0, hi = ncb - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (lpre[mid] <= f) lo = mid; else hi = mid - 1;
    }
    const int r = f - lpre[lo];
    const int cnt = min(lpre[lo + 1] - lpre[lo], d.bcap);
    if (r >= cnt) return;  // beyond the bucket (LE_E_CAPACITY latched by the binning)
    const int2* B = d.bucket + (size_t)(c0 + lo) * d.bcap;
    const int2 e = B[r];
    int rank = 0;
    for (int q = 0; q < cnt; ++q) rank += (B[q].x < e.x) ? 1 : 0;
    const int s = base + lpre[lo] + rank;
    if ((unsigned)s < (unsigned)d.n && (unsigned)e.y < (unsigned)d.n) {  // (else a latched error)
      ns = s;
      src = e.y;
      tg = e.x;
    }
  };
  struct St { double4 p; double v0, v1, v2, f0, f1, f2; };
  auto load = [&](int i) -> St {
    const double* V = d.vel[as];
    const double* F = d.frc[as];
    return St{reinterpret_cast<const double4*>(d.pos[ps])[i], V[i], V[np + i], V[2 * np + i],
              F[i], F[np + i], F[2 * np + i]};
  };
  auto store = [&](int ns, int tg, const St& v) {
    if (ns < 0) return;
    reinterpret_cast<double4*>(d.pos[pd])[ns] = v.p;
    double* V = d.vel[ad];
    double* F = d.frc[ad];
    V[ns] = v.v0; V[np + ns] = v.v1; V[2 * np + ns] = v.v2;
    F[ns] = v.f0; F[np + ns] = v.f1; F[2 * np + ns] = v.f2;
    d.tag[ad][ns] = tg;
    d.slot_of_tag[tg] = ns;
  };
  for (int f0 = threadIdx.x; f0 < agg; f0 += 2 * kBlock) {
    int ns0, src0, tg0, ns1, src1, tg1;
    locate_f(f0, ns0, src0, tg0);
    locate_f(f0 + kBlock, ns1, src1, tg1);
    const St a0 = load(src0), a1 = load(src1);  // (slot 0 for an empty lane: in bounds, not stored)
    store(ns0, tg0, a0);
    store(ns1, tg1, a1);
  }
}

__global__ void __launch_bounds__(kBlock) k_scan_permute(Dev d) { scan_permute_body(d, blockIdx.x); }

// Batched form: the blocks of one simulation are consecutive in the grid, so
// every block's predecessors were dispatched before it (the look-back waits
// only on them).
__global__ void __launch_bounds__(kBlock) k_scan_permute_b(Batch b) {
  int sm, bid;
  locate(b, blockIdx.x, sm, bid);
  scan_permute_body(stage_dev(b.dev[sm]), bid);
}

// Neighbour lists of radius r_list through the Lees-Edwards cell stencil.
// Rows that do not cross a gradient face use the 27-cell block with periodic
// x/z images.  A row reached across the top (bottom) face belongs to the image
// box shifted by +Delta (-Delta) along x; the cells of that row whose image
// overlaps [x_cell - r_list, x_cell + l_x + r_list] are the unwrapped indices
// k in [floor((ix l - r - sy Delta)/l), floor(((ix+1) l + r - sy Delta)/l)],
// at most four cells for l >= r (five with the rounding margin).  Each
// (cell, image) pair is visited once; with L > 2 r_list at most one image of
// a particle can lie within r_list, so no pair is counted twice.
//
// Tiles.  The particles of one tile (kTile consecutive cell-sorted slots)
// span a few cell rows.  For every covered row r, offset (dy, dz) and x-image
// sx, the cells the tile's stencils can reach in the neighbouring row form a
// contiguous slot range (a "piece").  The pieces are staged into LDS in a
// fixed order while they fit (kHalo positions).  With the halo layout,
// halo_slot / halo_code record the slot and image of every LDS position so
// that the force kernel can restage the same halo each step; the global
// layout keeps that table in LDS for the search alone.  Pairs whose partner
// is staged without image store its LDS index (16 bits, halo layout); the
// others store the partner's slot and image code in one 32-bit word.  Lists
// are padded with sentinels (LDS index kHalo, slot n) to whole batches.

// Element k of particle i in the blocked list layouts (see Dev).
__device__ __forceinline__ size_t idx8(int k, int i, int np) {
  return ((size_t)(k >> 3) * np + i) * 8 + (k & 7);
}
__device__ __forceinline__ size_t idx4(int k, int i, int np) {
  return ((size_t)(k >> 2) * np + i) * 4 + (k & 3);
}

// Unwrapped x-cell range [klo, khi] reached from cells xa..xb of a row across
// the gradient face with image sy (sy = 0: the plain periodic block).
__device__ __forceinline__ void x_range(const Dev& d, int xa, int xb, int sy, double Delta, double rmarg,
                                        int& klo, int& khi) {
  if (sy == 0) {
    klo = xa - 1; khi = xb + 1;
  } else {
    double sh = (double)sy * Delta;
    klo = (int)floor(((double)xa * d.lx - rmarg - sh) / d.lx);
    khi = (int)floor(((double)(xb + 1) * d.lx + rmarg - sh) / d.lx);
  }
}

__device__ __forceinline__ int cell_of_pos(const Dev& d, double4 p) {
  return (cell_index(p.z, d.inv_lz, d.nz) * d.ny + cell_index(p.y, d.inv_ly, d.ny)) * d.nx +
         cell_index(p.x, d.inv_lx, d.nx);
}

constexpr int kWaves = kTile / 64;

// Tile halo pieces: for each covered row r of the tile, offset (dy, dz) and
// x-image sx, the slot range of the neighbouring row reached by the tile.
// Fills the piece tables, assigns LDS offsets in a fixed order while they
// fit, stages the positions and records their slots.  Called by all threads.
struct Pieces {
  int start[kMaxRows * 9][kPieces];
  int count[kMaxRows * 9][kPieces];
  int off[kMaxRows * 9][kPieces];  // LDS offset, -1 if not staged
  int sx0[kMaxRows * 9];
  int npc[kMaxRows * 9];
  int code[kMaxRows * 9];          // image code (sy, sz) of the row; sx added per piece
  int nseg, ntot;
};

// Exact list test of one pair: the plain-definition displacement between
// particle i and slot q under image (sx, sy, sz), r^2 < r_list^2.
__device__ __forceinline__ bool in_list_exact(const Dev& d, double4 pi, double4 pj, double shx,
                                              double shy, double shz, double shd) {
  double dy = (pi.y - pj.y) - shy;
  double dx = ((pi.x - pj.x) - shd) - shx;
  double dz = (pi.z - pj.z) - shz;
  double r2 = dx * dx + dy * dy;
  r2 = r2 + dz * dz;
  return r2 < d.rlist2;
}

// Two threads per particle: thread t (half 0) and t + kTile (half 1) split
// each (dy, dz) range in two and write two sub-lists, which the force kernel
// reads as one sequence of batches.
template <int HALO, bool GL>
__device__ __forceinline__ void neighbors_body(const Dev& d, const int tile) {
  // staged positions: floats relative to the tile's first particle, image
  // added (8 spare entries: a batch may read up to 7 past the halo)
  __shared__ float hx[HALO + 8], hy[HALO + 8], hz[HALO + 8];
  __shared__ Pieces pc;
  // The staging table (one entry per piece: LDS offset, first slot, image
  // code; read only while the halo is staged) and the per-thread ring of list
  // entries (LDS indices of the halo layout, left as whole blocks; used only
  // by the scan after the staging barrier) share their LDS.
  union StageRing {
    struct {
      int off[kMaxRows * 9 * kPieces + 1];
      int start[kMaxRows * 9 * kPieces];
      int code[kMaxRows * 9 * kPieces];
    } st;
    uint16_t ring[GL ? 1 : 2 * kTile][16];
  };
  __shared__ __align__(16) StageRing sr;
  auto& lbuf = sr.ring;
  // with GL: the ring of list entries (slot and image code) of lists of
  // global slots, and the entry of every staged position (the lists need no
  // halo tables in global memory then)
  __shared__ __align__(16) uint32_t gslot[GL ? 2 * kTile : 1][kOtherBatch];
  __shared__ uint32_t hent[GL ? HALO + 8 : 1];
  Ctrl* c = d.ctrl;
  if (rebuild_off(d)) return;  // (the same two words for every wave)
  const int np = d.np, np2 = d.np2, K = d.K, n = d.n;
  const int s0 = tile * kTile;
  const int half = (int)(threadIdx.x / kTile);
  const int tl = (int)threadIdx.x - half * kTile;
  const int i = s0 + tl;
  const int v = half * np + i;  // this thread's sub-list
  const bool valid = i < n;
  const int pn = c->pos_cur, an = c->aux_cur;  // sorted buffers of the new state
  const double4* P = reinterpret_cast<const double4*>(d.pos[pn]);
  const double Delta = c->Delta;
  const double rmarg = d.rlist * (1.0 + 1e-12) + 1e-12 * (d.Lx + d.Ly + d.Lz);

  // ---- tile geometry (every thread: the cells of the tile's first and last
  // particle, read through the scalar cache)
  const int c_first = cell_of_pos(d, P[s0]), c_last = cell_of_pos(d, P[min(s0 + kTile, n) - 1]);
  const int row_first = c_first / d.nx, nrows = c_last / d.nx - row_first + 1;
  const bool staged_ok = nrows <= kMaxRows;
  if (threadIdx.x == 0) {
    pc.nseg = 0;  // (no piece staged unless the first fits)
    pc.ntot = 0;
  }
  // ---- pieces: one thread per (covered row, dz, dy)
  const int ncombo = staged_ok ? nrows * 9 : 0;
  for (int t = threadIdx.x; t < ncombo; t += blockDim.x) {
    int r = t / 9, rem = t % 9;
    int dzc = rem / 3 - 1, dyc = rem % 3 - 1;
    int row = row_first + r;
    int iy = row % d.ny, iz = row / d.ny;
    int xa = (r == 0) ? c_first % d.nx : 0;
    int xb = (r == nrows - 1) ? c_last % d.nx : d.nx - 1;
    int jz = iz + dzc, sz = jz < 0 ? -1 : (jz >= d.nz ? 1 : 0);
    jz -= sz * d.nz;
    int jy = iy + dyc, sy = jy < 0 ? -1 : (jy >= d.ny ? 1 : 0);
    jy -= sy * d.ny;
    int klo, khi;
    x_range(d, xa, xb, sy, Delta, rmarg, klo, khi);
    int sxa = floor_div(klo, d.nx), sxb = floor_div(khi, d.nx);
    int npc = sxb - sxa + 1;
    pc.sx0[t] = sxa;
    pc.code[t] = (sy + 1) | ((sz + 1) << 2);
    pc.npc[t] = npc <= kPieces ? npc : 0;  // 0: not staged (too many images)
    const int rowbase = (jz * d.ny + jy) * d.nx;
    for (int q = 0; q < kPieces; ++q) {
      pc.start[t][q] = 0;
      pc.count[t][q] = 0;
      if (q < pc.npc[t]) {
        int sx = sxa + q;
        int ka = max(klo, sx * d.nx), kb = min(khi, sx * d.nx + d.nx - 1);
        int c0 = rowbase + (ka - sx * d.nx), c1 = rowbase + (kb - sx * d.nx);
        pc.start[t][q] = d.cell_start[c0];
        pc.count[t][q] = d.cell_start[c1 + 1] - d.cell_start[c0];
      }
    }
  }
  __syncthreads();
  // ---- LDS offsets in a fixed order (prefix sum over the pieces); pieces that
  // do not fit stay global.  One piece per thread of the first kWaves waves.
  {
    static_assert(kMaxRows * 9 * kPieces <= kTile, "one piece per thread of the first kTile");
    __shared__ int wsum[kWaves];
    const int npieces = ncombo * kPieces;
    const int e = (int)threadIdx.x;
    const bool pe = e < npieces;
    const int t = pe ? e / kPieces : 0, q = e % kPieces;
    const bool real = pe && q < pc.npc[t];
    const int cnt = real ? pc.count[t][q] : 0;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    int incl = cnt;
    for (int o = 1; o < 64; o <<= 1) {
      const int u = __shfl_up(incl, o, 64);
      if (lane >= o) incl += u;
    }
    if (lane == 63 && wv < kWaves) wsum[wv] = incl;
    __syncthreads();
    for (int w2 = 0; w2 < kWaves; ++w2)
      if (w2 < wv) incl += wsum[w2];
    // a piece is staged iff it ends within the halo; the staged set is a
    // prefix of the pieces (the running offsets only grow).  The staging
    // table is that prefix, one entry per piece in order (empty ones too:
    // the search below skips them), written by the piece's own thread; the
    // last piece that fits records the prefix's length and size.
    if (pe) {
      const int start_off = incl - cnt;
      const bool fits = incl <= HALO;
      pc.off[t][q] = (real && fits) ? start_off : -1;
      sr.st.off[e] = start_off;
      sr.st.start[e] = real ? pc.start[t][q] : 0;
      sr.st.code[e] = real ? pack_img(pc.sx0[t] + q, (pc.code[t] & 3) - 1, (pc.code[t] >> 2) - 1) : 0;
      bool next_fits = false;
      if (e + 1 < npieces) {
        const int t1 = (e + 1) / kPieces, q1 = (e + 1) % kPieces;
        next_fits = incl + (q1 < pc.npc[t1] ? pc.count[t1][q1] : 0) <= HALO;
      }
      if (fits && !next_fits) {
        pc.nseg = e + 1;
        pc.ntot = incl;
      }
    }
    __syncthreads();
    if (threadIdx.x == 0) d.tile_nstage[tile] = pc.ntot;
  }
  // ---- stage positions and record their slots (flat, kStageLoads loads in
  // flight per thread: the search halo in one round)
  const double4 org = P[s0];
  {
    const int tot = pc.ntot, nseg = pc.nseg;
    constexpr int kStageLoads = 6;
    for (int h0 = threadIdx.x; h0 < tot; h0 += kStageLoads * blockDim.x) {
      int slot[kStageLoads], code[kStageLoads];
#pragma unroll
      for (int u = 0; u < kStageLoads; ++u) {
        int h = h0 + u * blockDim.x;
        slot[u] = n;
        code[u] = 0;
        if (h < tot) {
          int lo = 0, hi = nseg - 1;  // last segment with s_off <= h
          while (lo < hi) {
            int mid = (lo + hi + 1) >> 1;
            if (sr.st.off[mid] <= h) lo = mid; else hi = mid - 1;
          }
          slot[u] = sr.st.start[lo] + (h - sr.st.off[lo]);
          code[u] = sr.st.code[lo];
        }
      }
      double4 pj[kStageLoads];
#pragma unroll
      for (int u = 0; u < kStageLoads; ++u) pj[u] = P[slot[u]];
#pragma unroll
      for (int u = 0; u < kStageLoads; ++u) {
        const int h = h0 + u * blockDim.x;
        // written unconditionally (past the halo: a spare entry) so that the
        // loads above are not sunk into the condition one by one
        const int hw = h < tot ? h : HALO + 7;
        int sx, sy, sz;
        unpack_img((uint8_t)code[u], sx, sy, sz);
        hx[hw] = (float)((pj[u].x + ((double)sy * Delta + (double)sx * d.Lx)) - org.x);
        hy[hw] = (float)((pj[u].y + (double)sy * d.Ly) - org.y);
        hz[hw] = (float)((pj[u].z + (double)sz * d.Lz) - org.z);
        if constexpr (GL) {
          hent[hw] = og_entry((uint32_t)slot[u], (uint8_t)code[u]);
        } else if (h < tot) {
          d.halo_slot[(size_t)tile * kHalo + h] = slot[u];
          d.halo_code[(size_t)tile * kHalo + h] = (uint8_t)code[u];
        }
      }
    }
  }

  __syncthreads();

  // ---- scan: each lane walks its own stencil.  For each (dy, dz) the x-cells
  // the particle reaches in that row form one contiguous LDS range (the row's
  // x-image pieces are staged back to back, images already added), so a lane
  // tests [a, b) with eight candidates per batch, the particle's two threads
  // taking alternate batches (each sub-list then holds partners from all
  // over the row: fewer padding entries and gathers spread alike); the wave
  // runs to its longest range.  Lanes whose row was not staged walk the cells
  // in global memory with the exact test instead.
  const double4 pi = P[valid ? i : s0];
  const float pix = (float)(pi.x - org.x), piy = (float)(pi.y - org.y), piz = (float)(pi.z - org.z);
  const int ix = cell_index(pi.x, d.inv_lx, d.nx);
  const int iy = cell_index(pi.y, d.inv_ly, d.ny);
  const int iz = cell_index(pi.z, d.inv_lz, d.nz);
  const int rt = (iz * d.ny + iy) - row_first;  // tile row of the particle
  const bool row_staged = valid && staged_ok && rt >= 0 && rt < nrows;
  int self_h = -1;  // LDS position of the particle itself (plain image)
  if (row_staged) {
    const int t = rt * 9 + 4;  // dz = dy = 0
    const int q = -pc.sx0[t];  // sx = 0
    if (q >= 0 && q < pc.npc[t] && pc.off[t][q] >= 0) self_h = i - pc.start[t][q] + pc.off[t][q];
  }
  const float tlo = d.nb_lo, thi = d.nb_hi;
  const size_t hbase = (size_t)tile * kHalo;
  int npl = 0, nog = 0;
  // one global-list entry (og_entry: slot and image code in one word): with
  // GL into the lane's ring, a completed block of four leaving as one 16-byte
  // store; otherwise (rows beyond the halo of a halo-layout list) straight to
  // global memory
  auto og_append = [&](uint32_t e) {
    if constexpr (GL) {
      gslot[threadIdx.x][nog & 3] = e;
      ++nog;
      if ((nog & 3) == 0 && nog <= K) {
        const size_t b = (size_t)((nog >> 2) - 1) * np2 + v;
        reinterpret_cast<uint4*>(d.nlo)[b] = *reinterpret_cast<const uint4*>(gslot[threadIdx.x]);
      }
    } else {
      if (nog < K) d.nlo[idx4(nog, v, np2)] = e;
      ++nog;
    }
  };
  for (int c9 = 0; c9 < 9; ++c9) {
    const int dzc = c9 / 3 - 1, dyc = c9 % 3 - 1;
    int jz = iz + dzc, sz = jz < 0 ? -1 : (jz >= d.nz ? 1 : 0);
    jz -= sz * d.nz;
    int jy = iy + dyc, sy = jy < 0 ? -1 : (jy >= d.ny ? 1 : 0);
    jy -= sy * d.ny;
    int klo, khi;
    x_range(d, ix, ix, sy, Delta, rmarg, klo, khi);
    const int rowbase = (jz * d.ny + jy) * d.nx;
    int a = 0, b = 0;
    bool walk_global = valid;
    if (row_staged) {
      const int t = rt * 9 + c9;
      const int sxa = floor_div(klo, d.nx), sxb = floor_div(khi, d.nx);
      const int qa = sxa - pc.sx0[t], qb = sxb - pc.sx0[t];
      // staged pieces form a prefix, so the last one staged implies the rest
      if (qa >= 0 && qb < pc.npc[t] && pc.off[t][qb] >= 0) {
        a = d.cell_start[rowbase + (klo - sxa * d.nx)] + (pc.off[t][qa] - pc.start[t][qa]);
        b = d.cell_start[rowbase + (khi - sxb * d.nx) + 1] + (pc.off[t][qb] - pc.start[t][qb]);
        // the two threads of the particle take alternate batches of the range
        a += 8 * half;
        walk_global = false;
      }
    }
    int wlen = b - a;
    for (int o = 32; o > 0; o >>= 1) wlen = max(wlen, __shfl_xor(wlen, o, 64));
    wlen = __builtin_amdgcn_readfirstlane(wlen);
    const int sq = (c9 == 4) ? self_h : -1;
    for (int j0 = 0; j0 < wlen; j0 += 16) {
      const int h0 = a + j0;
      // candidates past the lane's range are read (in bounds) and masked off
      const int lim = b - h0;
      unsigned keep = lim >= 8 ? 0xffu : (lim > 0 ? (1u << lim) - 1u : 0u);
      if (sq >= h0 && sq < h0 + 8) keep &= ~(1u << (sq - h0));
      const int hc = min(h0, HALO);
      unsigned m_in = 0u, m_band = 0u;
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const float dx = pix - hx[hc + u];
        const float dy = piy - hy[hc + u];
        const float dz = piz - hz[hc + u];
        const float r2 = __builtin_fmaf(dz, dz, __builtin_fmaf(dy, dy, dx * dx));
        m_in |= (r2 < tlo ? 1u : 0u) << u;
        m_band |= (r2 < thi ? 1u : 0u) << u;
      }
      m_in &= keep;
      m_band &= keep & ~m_in;
      while (m_band) {  // rare: FP32 r^2 within the rounding band of r_list^2
        const int u = __builtin_ctz(m_band);
        m_band &= m_band - 1u;
        const int h = h0 + u;
        int q2;
        uint8_t c2;
        if constexpr (GL) {
          q2 = (int)(hent[h] & kSlotMask);
          c2 = (uint8_t)(hent[h] >> kSlotBits);
        } else {
          q2 = d.halo_slot[hbase + h];
          c2 = d.halo_code[hbase + h];
        }
        int sx2, sy2, sz2;
        unpack_img(c2, sx2, sy2, sz2);
        if (in_list_exact(d, pi, P[q2], (double)sx2 * d.Lx, (double)sy2 * d.Ly, (double)sz2 * d.Lz,
                          (double)sy2 * Delta))
          m_in |= 1u << u;
      }
      if constexpr (GL) {
        // lists without a force-time halo: the partner's slot and image code
        while (m_in) {
          const int u = __builtin_ctz(m_in);
          m_in &= m_in - 1u;
          og_append(hent[h0 + u]);
        }
      } else {
        // append the accepted LDS indices into a ring of 16 per lane: every
        // candidate is written at the next free entry and the count advances
        // only for accepted ones (a rejected one is overwritten by the next
        // write); a completed block of 8 leaves as one 16-byte store
        int nn = npl;
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          lbuf[threadIdx.x][nn & 15] = (uint16_t)(h0 + u);
          nn += (int)((m_in >> u) & 1u);
        }
        if ((nn >> 3) != (npl >> 3)) {
          const int blk = npl >> 3;
          if ((blk + 1) * 8 <= K)
            reinterpret_cast<uint4*>(d.nl16)[(size_t)blk * np2 + v] =
                *reinterpret_cast<const uint4*>(&lbuf[threadIdx.x][(blk & 1) * 8]);
        }
        npl = nn;
      }
    }
    if (walk_global) {
      // this particle's cells of the row, read from global memory; the two
      // threads of the particle take the lower and the upper cells
      const int kmid = klo + (khi - klo) / 2;
      const int ka = half == 0 ? klo : kmid + 1, kb = half == 0 ? kmid : khi;
      for (int k = ka; k <= kb; ++k) {
        const int sx = floor_div(k, d.nx);
        const int cell = rowbase + (k - sx * d.nx);
        const bool plain = (sx == 0 && sy == 0 && sz == 0);
        const uint8_t code = pack_img(sx, sy, sz);
        for (int q = d.cell_start[cell]; q < d.cell_start[cell + 1]; ++q) {
          if (plain && q == i) continue;
          if (in_list_exact(d, pi, P[q], (double)sx * d.Lx, (double)sy * d.Ly, (double)sz * d.Lz,
                            (double)sy * Delta)) {
            og_append(og_entry((uint32_t)q, code));
          }
        }
      }
    }
  }
  {
    // the second sub-list's last, partial block (still in its thread's ring)
    // moves to the end of the first: the two sub-lists then carry one padding
    // instead of two (the force kernels read them as one sequence).  Entries
    // of the halo layout's rows beyond the halo went straight to global
    // memory and stay where they are.
    // entries of the partial block | its ring half << 8, where the staged y
    // coordinates were (every wave has left the scan after this barrier)
    int* tail = reinterpret_cast<int*>(hy);
    __syncthreads();
    if (half == 1)
      tail[tl] = GL ? (nog & (kOtherBatch - 1)) : ((npl & (kPlainBatch - 1)) | (((npl >> 3) & 1) << 8));
    __syncthreads();
    const int r = tail[tl] & 0xff;
    const int pt = (int)threadIdx.x + kTile;  // the particle's second thread
    if (half == 0) {
      if constexpr (GL) {
        for (int k = 0; k < r; ++k) og_append(gslot[pt][k]);
      } else {
        const int src = (tail[tl] >> 8) * 8;
        for (int k = 0; k < r; ++k) {
          lbuf[threadIdx.x][npl & 15] = lbuf[pt][src + k];
          ++npl;
          const int blk = (npl >> 3) - 1;  // completed by this entry
          if ((npl & 7) == 0 && (blk + 1) * 8 <= K)
            reinterpret_cast<uint4*>(d.nl16)[(size_t)blk * np2 + v] =
                *reinterpret_cast<const uint4*>(&lbuf[threadIdx.x][(blk & 1) * 8]);
        }
      }
    } else {
      if constexpr (GL) nog -= r; else npl -= r;
    }
  }
  {  // telemetry (entries per particle, both sub-lists): one atomic per block
    __shared__ int wmax[2 * kTile / 64];
    // the counts of the second halves go where the staged x coordinates
    // were: every wave has left the scan after this barrier
    __syncthreads();
    int* cnt1 = reinterpret_cast<int*>(hx);
    if (half == 1) cnt1[tl] = npl + nog;
    __syncthreads();
    int mx = half == 0 ? npl + nog + cnt1[tl] : 0;
    for (int o = 32; o > 0; o >>= 1) mx = max(mx, __shfl_xor(mx, o, 64));
    if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = mx;
    __syncthreads();
    if (threadIdx.x == 0) {
      for (int w = 1; w < 2 * kTile / 64; ++w) mx = max(mx, wmax[w]);
      atomicMax(&d.flags->max_nb_slot[(tile % kSlots) * kLineInts], mx);
    }
  }
  if (!valid) return;
  int npl_p = (npl + kPlainBatch - 1) / kPlainBatch * kPlainBatch;
  int nog_p = (nog + kOtherBatch - 1) / kOtherBatch * kOtherBatch;
  if (npl_p > K || nog_p > K) {
    latch(d.flags, LE_E_CAPACITY);
    npl_p = nog_p = 0;
  } else {
    if constexpr (!GL) {
      if (npl < npl_p) {  // pad and flush the partial block
        const int blk = npl >> 3;
        for (int r = npl; r < npl_p; ++r) lbuf[threadIdx.x][r & 15] = (uint16_t)kHalo;
        reinterpret_cast<uint4*>(d.nl16)[(size_t)blk * np2 + v] =
            *reinterpret_cast<const uint4*>(&lbuf[threadIdx.x][(blk & 1) * 8]);
      }
    }
    const uint8_t zero = pack_img(0, 0, 0);
    while (nog < nog_p) og_append(og_entry((uint32_t)n, zero));  // sentinel entries up to a whole block
  }
  d.n_plain[v] = npl_p;
  d.n_og[v] = nog_p;
  if (d.chain_len > 0 && half == 0) {
    int tg_ = d.tag[an][i];
    int lo = -1, hi = -1;
    if (tg_ < d.n_bonded) {
      int kk = tg_ % d.chain_len;
      if (kk > 0) lo = d.slot_of_tag[tg_ - 1];
      if (kk < d.chain_len - 1) hi = d.slot_of_tag[tg_ + 1];
    }
    d.bond[i] = lo;
    d.bond[np + i] = hi;
  }
}

template <int HALO, bool GL>
__global__ void __launch_bounds__(2 * kTile) k_neighbors(Dev d) {
  neighbors_body<HALO, GL>(d, xcd_block(d.ntiles));
}

constexpr int kSpreadRun = 4;  // consecutive tiles per run of the batched list search

// Batched form: only the members that rebuild at this step have work, so the
// blocks are spread over the XCDs in short runs (xcd_spread) rather than in
// one contiguous range per XCD; then the tile is located.
template <int HALO, bool GL>
__global__ void __launch_bounds__(2 * kTile) k_neighbors_b(Batch b) {
  int sm, tile;
  locate(b, xcd_spread<kSpreadRun>((int)blockIdx.x, (int)gridDim.x), sm, tile);
  neighbors_body<HALO, GL>(stage_dev(b.dev[sm]), tile);
}

// ---------------------------------------------------------- integrator
// Block maximum of |c|^2 into one of the kSlots words; called by every
// thread of a block of exactly NTH threads (the LDS array holds one entry per
// wave of that block; launches pass the kernel's own block size).
template <int NTH>
__device__ __forceinline__ void vmax_commit(const Dev& d, double v2, int lb) {
  static_assert(NTH % 64 == 0 && NTH <= 1024, "whole waves, at most 16");
  __shared__ double wm[NTH / 64];
  double m = wave_max(v2);
  if ((threadIdx.x & 63) == 0) wm[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < NTH / 64; ++w) m = fmax(m, wm[w]);
    atomicMax(&d.vmax[(lb % kSlots) * kLineU64], (unsigned long long)__double_as_longlong(m));
  }
}

// Sum the per-block stress partials (fixed order) and write the stress
// -(K + W)/V, or with virial_only the pair virial W, into out6.  Called by one
// whole block of kBlock threads.
__device__ void reduce_partials(const Dev& d, double* out6, bool virial_only) {
  __shared__ double red[kBlock / 64][kStressComps];
  double acc[kStressComps];
#pragma unroll
  for (int k = 0; k < kStressComps; ++k) acc[k] = 0.0;
  for (int b = threadIdx.x; b < d.nblocks; b += blockDim.x) {
#pragma unroll
    for (int k = 0; k < kStressComps; ++k) acc[k] += d.partials[b * kStressComps + k];
  }
  int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < kStressComps; ++k) {
    double v = acc[k];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if (lane == 0) red[wid][k] = v;
  }
  __syncthreads();
  if (threadIdx.x < 6) {
    double kin = 0.0, vir = 0.0;
    for (int w = 0; w < kBlock / 64; ++w) {
      kin += red[w][threadIdx.x];
      vir += red[w][6 + threadIdx.x];
    }
    out6[threadIdx.x] = virial_only ? vir : -(kin + vir) * d.inv_vol;
  }
}

// First half-kick and drift from a state with full-step velocities:
// u += dt/(2m) F ; x_new = x + dt u (into the other position buffer).  The
// step is advanced by the next control kernel.
__device__ __forceinline__ void kick_drift_body(const Dev& d, int bid) {
  __shared__ int skip;
  Ctrl* c = d.ctrl;
  if (threadIdx.x == 0) skip = d.flags->status;
  __syncthreads();
  if (skip) return;
  int i = bid * kBlock + threadIdx.x;
  const int np = d.np;
  double v2 = 0.0;
  if (i < d.n) {
    const int pc = c->pos_cur, ac = c->aux_cur;
    double4 p = reinterpret_cast<const double4*>(d.pos[pc])[i];
    double* U = d.vel[ac];
    const double* F = d.frc[ac];
    double ux = U[i] + d.h * F[i];
    double uy = U[np + i] + d.h * F[np + i];
    double uz = U[2 * np + i] + d.h * F[2 * np + i];
    double cx = ux - d.c_sr * (p.y - 0.5 * d.Ly);
    v2 = cx * cx + uy * uy + uz * uz;
    U[i] = ux; U[np + i] = uy; U[2 * np + i] = uz;
    double4 q;
    q.x = p.x + d.dt * (ux + d.drift_sr * (p.y - 0.5 * d.Ly));
    q.y = p.y + d.dt * uy;
    q.z = p.z + d.dt * uz;
    q.w = p.w;
    reinterpret_cast<double4*>(d.pos[1 - pc])[i] = q;
    if (!(isfinite(q.x) && isfinite(q.y) && isfinite(q.z))) latch(d.flags, LE_E_NONFINITE);
  }
  vmax_commit<kBlock>(d, v2, bid);
}

__global__ void __launch_bounds__(kBlock) k_kick_drift(Dev d) { kick_drift_body(d, blockIdx.x); }

__global__ void __launch_bounds__(kBlock) k_kick_drift_b(Batch b) {
  int sm, bid;
  locate(b, blockIdx.x, sm, bid);
  kick_drift_body(stage_dev(b.dev[sm]), bid);
}

// ---------------------------------------------------------- force kernel
template <bool VIR>
__device__ __forceinline__ void add_pair(double f, double dx, double dy, double dz, double& fx,
                                         double& fy, double& fz, double* w) {
  fx = fma(f, dx, fx); fy = fma(f, dy, fy); fz = fma(f, dz, fz);
  if (VIR) {
    double ax = f * dx, ay = f * dy, az = f * dz;
    w[0] = fma(dx, ax, w[0]); w[1] = fma(dy, ay, w[1]); w[2] = fma(dz, az, w[2]);
    w[3] = fma(dx, ay, w[3]); w[4] = fma(dx, az, w[4]); w[5] = fma(dy, az, w[5]);
  }
}

// Scalar LJ force factor f (force on i = f d) for r^2 = r2, zero outside the
// cutoff.  Branch-free so that the candidates of one batch are independent
// instruction streams the compiler can interleave.  With CAP (FP64 only) the
// magnitude |f| r is limited to cap: |f| <= cap / r.
template <bool MIXED, bool CAP = false>
__device__ __forceinline__ double lj_masked(double r2, double rc2, double sig2, double eps24,
                                            double cap = 0.0) {
  static_assert(!(MIXED && CAP), "the capped force law is FP64");
  const bool in = r2 < rc2;
  if (MIXED) {
    float r2f = (float)r2;
    float inv = __builtin_amdgcn_rcpf(r2f);
    inv = inv * (2.0f - r2f * inv);  // one Newton step: ~1 ulp
    float s2 = (float)sig2 * inv;
    float s6 = s2 * s2 * s2;
    float f = (float)eps24 * s6 * (2.0f * s6 - 1.0f) * inv;
    return in ? (double)f : 0.0;
  } else {
    double inv = __builtin_amdgcn_rcp(r2);
    double e = fma(-r2, inv, 1.0);
    inv = fma(inv, e, inv);
    e = fma(-r2, inv, 1.0);
    inv = fma(inv, e, inv);
    double s2 = sig2 * inv;
    double s6 = s2 * s2 * s2;
    double f = s6 * fma(2.0 * eps24, s6, -eps24) * inv;  // 24 eps s6 (2 s6 - 1) / r^2
    if (CAP) {
      const double lim = cap / sqrt(r2);
      f = fmin(fmax(f, -lim), lim);
    }
    return in ? f : 0.0;
  }
}

// Lees-Edwards nearest-image displacement a - b (the integers by rounding;
// valid for bonded beads, which are far closer than half a box).
__device__ __forceinline__ void near_disp(const Dev& d, double4 a, double4 b, double Delta, double& dx,
                                          double& dy, double& dz) {
  const double dy0 = a.y - b.y;
  const double sy = rint(dy0 / d.Ly);
  dy = dy0 - sy * d.Ly;
  const double dx0 = (a.x - b.x) - sy * Delta;
  const double sx = rint(dx0 / d.Lx);
  dx = dx0 - sx * d.Lx;
  const double dz0 = a.z - b.z;
  const double sz = rint(dz0 / d.Lz);
  dz = dz0 - sz * d.Lz;
}

// Cosine angle term (Eq. angle) read as V = k (1 + cos theta), minimum at a
// straight chain: theta the angle between b1 = x_a - x_j and b2 = x_b - x_j at
// the middle bead j.  Forces on the two ends (F_j = -(F_a + F_b)):
//   F_a = -k [b2 / (l1 l2) - cos(theta) b1 / l1^2],  F_b likewise.
__device__ __forceinline__ void angle_cos(const double b1[3], const double b2[3], double k, double Fa[3],
                                          double Fb[3]) {
  const double l11 = b1[0] * b1[0] + b1[1] * b1[1] + b1[2] * b1[2];
  const double l22 = b2[0] * b2[0] + b2[1] * b2[1] + b2[2] * b2[2];
  const double l12 = sqrt(l11) * sqrt(l22);
  const double c = (b1[0] * b2[0] + b1[1] * b2[1] + b1[2] * b2[2]) / l12;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    Fa[a] = -k * (b2[a] / l12 - c * b1[a] / l11);
    Fb[a] = -k * (b1[a] / l12 - c * b2[a] / l22);
  }
}

// DPD pair terms (Eqs. dissipative, random, omega) on particle i from one
// partner: d = x_i - x_j(image), v = u_i - u_j(image) (the image's streaming
// velocity already removed), r2 = |d|^2.  Adds f d with
// f = [-gamma w^2 (d.v / r) + sqrt(24 gamma kT / dt) w theta_ij] / r,
// w = 1 - r / r_c, zero at and beyond r_c.  theta_ij is word 0 of the Philox
// block with counter (step, smaller tag, larger tag), so both members of the
// pair draw the same number and their forces cancel.
__device__ __forceinline__ void dpd_pair(const Dev& d, uint32_t s_lo, uint32_t s_hi, int ti, int tj,
                                         double vx, double vy, double vz, double dx, double dy,
                                         double dz, double r2, double& ax, double& ay, double& az) {
  const bool in = r2 < d.dpd_rc2;
  // 1/r from the hardware reciprocal square root and two Newton steps
  // (within 2 ulp of the quotient), then r = r2 / r: the IEEE square root and
  // division cost the pair about 14 instructions more
  const double h = 0.5 * r2;
  double ir = __builtin_amdgcn_rsq(r2);
  ir = ir * fma(-h * ir, ir, 1.5);
  ir = ir * fma(-h * ir, ir, 1.5);
  const double r = r2 * ir;
  const double wgt = 1.0 - r * d.dpd_inv_rc;
  double ev = dx * vx + dy * vy;
  ev = (ev + dz * vz) * ir;
  uint32_t c[4] = {s_lo, s_hi, (uint32_t)min(ti, tj), (uint32_t)max(ti, tj)};
  philox(c, d.seed_lo, d.dpd_key_hi);
  double f = (-d.dpd_gamma * wgt * wgt * ev + d.dpd_pref * wgt * u01c(c[0])) * ir;
  f = in ? f : 0.0;
  ax = fma(f, dx, ax); ay = fma(f, dy, ay); az = fma(f, dz, az);
}

// Block reduction of 12 per-thread sums into partials[block][12] (fixed
// order: wave butterflies, then waves in index order).  Called by every thread
// of a block of exactly NTH threads (one LDS row per wave of that block).
template <int NTH>
__device__ __forceinline__ void block_partials(double* vals, double* out, int lb,
                                               int nwrite = kStressComps) {
  static_assert(NTH % 64 == 0 && NTH <= 1024, "whole waves, at most 16");
  __shared__ double red[NTH / 64][kStressComps];
  int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < kStressComps; ++k) {
    double v = vals[k];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if (lane == 0) red[wid][k] = v;
  }
  __syncthreads();
  if (threadIdx.x < nwrite) {
    double s = 0.0;
    for (int w = 0; w < NTH / 64; ++w) s += red[w][threadIdx.x];
    out[lb * kStressComps + threadIdx.x] = s;
  }
}

// One evaluation of the conservative force for every particle, and then,
// depending on MODE:
//   kForcesOnly  write F^c in tag order (+ kinetic and virial partials)
//   kInitForce   F = F^c + Langevin(u) of the current step into frc
//   kStepLast    F as above from the half-step velocity, u += dt/(2m) F
//   kStepFused   as kStepLast, then the next half-kick and drift
//   kDpdForce    F = F^c + DPD pair terms of the current (half-step)
//                velocities into frc; k_integrate then moves the particles
//                (velocities of partners must not change while it runs)
// Langevin force (Eq. langevin on the peculiar velocity, Eq. vi):
//   F = F^c - gamma m c + sqrt(24 gamma m kT / dt) theta,  c = u - gamma_dot (y - L_y/2) e_x
// (with the friction on the lab velocity, c = u of the image inside the box).
// With the LDS halo the block has kForceTPP threads per particle: threads
// t, t + kTile, ... take every kForceTPP-th batch of the particle's list (more
// waves per CU for the same LDS), and hand their partial sums to the first
// through LDS before the epilogue.  Without the halo the launch bound of four
// tiles per block makes the compiler keep fewer registers (more waves; DPD
// 138 -> 132 us); the launch itself uses one tile.
template <int MODE, bool MIXED, bool BONDS, bool SAMPLE, bool STAGED, bool CAP>
__device__ __forceinline__ void force_body(const Dev& d, const int lb, double* __restrict__ f_out) {
  static_assert(!CAP || (!STAGED && !MIXED && MODE != kDpdForce), "capped forces: FP64, global layout");
  constexpr bool VIR = SAMPLE || (MODE == kForcesOnly);
  constexpr bool DPD = MODE == kDpdForce;
  static_assert(!DPD || !STAGED, "DPD partners come from global memory");
  constexpr int kH = STAGED ? kHalo + 1 : 1;  // no halo: every partner from global memory
  constexpr int TPP = STAGED ? kForceTPP : kGlobalTPP;  // threads per particle
  constexpr int kTh = TPP * kTile;                      // threads per block
  static_assert(STAGED || TPP <= 2, "global layout: at most one thread per sub-list");
  static_assert(!STAGED || 3 * kH >= kTile * 9 * (kForceTPP - 1), "the halo holds the partial-sum exchange");
  __shared__ double hbuf[3 * kH];
  double* const hx = hbuf;
  double* const hy = hbuf + kH;
  double* const hz = hbuf + 2 * kH;
  __shared__ int skip;
  Ctrl* c = d.ctrl;
  if (threadIdx.x == 0) skip = d.flags->status;
  __syncthreads();
  if (skip) return;
  const int half = TPP > 1 ? (int)(threadIdx.x / kTile) : 0;
  const int tl = (int)threadIdx.x - half * kTile;  // particle within the tile
  const int i = lb * kTile + tl;
  const bool valid = i < d.n;
  const int np = d.np;
  const int pc = c->pos_cur, ac = c->aux_cur;
  const double Delta = c->Delta;
  const int W = c->wraps;
  const double4* P = reinterpret_cast<const double4*>(d.pos[pc]);
  // Per-particle data and the first list blocks are requested before and
  // during the halo staging so that their latency overlaps it (loads use a
  // clamped index; values of invalid lanes are never used).
  const int ic = valid ? i : 0;
  const int np2 = d.np2;
  const double4 pi_ld = P[ic];
  const int npl0_ld = STAGED ? d.n_plain[ic] : 0, npl1_ld = STAGED ? d.n_plain[np + ic] : 0;
  const double* Uv = d.vel[ac];
  const double u0_ld = Uv[ic], u1_ld = Uv[np + ic], u2_ld = Uv[2 * np + ic];
  const int tag_ld = d.tag[ac][ic];
  const uint4* __restrict__ l8 = reinterpret_cast<const uint4*>(d.nl16) + ic;
  const int last_blk = d.K / kPlainBatch - 1;
  const int nb0 = STAGED ? npl0_ld / kPlainBatch : 0;
  // offset (in uint4) of batch b of the particle's two sub-lists read as one
  // sequence (sub-list 0, then sub-list 1)
  auto boff = [&](int b) -> size_t {
    const int sub = b < nb0 ? 0 : 1;
    const int blk = min(b - sub * nb0, last_blk);
    return (size_t)blk * np2 + (size_t)sub * np;
  };
  uint4 t0 = make_uint4(0u, 0u, 0u, 0u), t1 = t0;
  // Stage the tile's halo: the slots recorded at the last build with their
  // current positions, each shifted by its periodic / Lees-Edwards image
  // (sy Delta + sx L_x, sy L_y, sz L_z; the x image absorbs the offset's
  // wraps since the build).  A partner's displacement is then x_i - x_h.  All
  // slot loads, then all position loads, are in flight together.
  if (STAGED) {
    const int nst = d.tile_nstage[lb];
    const int* hs = d.halo_slot + (size_t)lb * kHalo;
    const uint8_t* hc = d.halo_code + (size_t)lb * kHalo;
    constexpr int U = kHalo / kTh;
    int slot[U];
    uint8_t code[U];
    const int nsent = d.n;
#pragma unroll
    for (int u = 0; u < U; ++u) {
      // always load from an index inside this tile's table, then select the value
      int h = threadIdx.x + u * kTh;
      int hh = h < nst ? h : 0;
      int sv = hs[hh];
      uint8_t cv = hc[hh];
      slot[u] = (h < nst) ? sv : nsent;
      code[u] = (h < nst) ? cv : pack_img(0, 0, 0);
    }
    t0 = l8[boff(half)];
    t1 = l8[boff(half + kForceTPP)];
    // every position is loaded and written (past nst: the sentinel slot, an
    // unused LDS entry), so that no load is sunk into a condition and all of
    // them are in flight together
    double4 pj[U];
#pragma unroll
    for (int u = 0; u < U; ++u) pj[u] = P[slot[u]];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int h = threadIdx.x + u * kTh;
      int sx, sy, sz;
      unpack_img(code[u], sx, sy, sz);
      sx += sy * W;
      hx[h] = pj[u].x + ((double)sy * Delta + (double)sx * d.Lx);
      hy[h] = pj[u].y + (double)sy * d.Ly;
      hz[h] = pj[u].z + (double)sz * d.Lz;
    }
    if (threadIdx.x == 0) { hx[kHalo] = 1e100; hy[kHalo] = 1e100; hz[kHalo] = 1e100; }
    __syncthreads();
  }
  double fx = 0.0, fy = 0.0, fz = 0.0;
  double gx = 0.0, gy = 0.0, gz = 0.0;  // DPD pair terms (kept out of the virial)
  double w[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  const double4 pi = valid ? pi_ld : make_double4(0.0, 0.0, 0.0, 0.0);
  const uint32_t st_lo = (uint32_t)(uint64_t)c->step, st_hi = (uint32_t)((uint64_t)c->step >> 32);
  const double4* __restrict__ VT = reinterpret_cast<const double4*>(d.vt);
  if (valid) {
    const double rc2 = d.rc2, sig2 = d.sig2, eps24 = d.eps24;
    // staged partners (already shifted to their image): the particle's two
    // sub-lists read as one sequence of batches of 8, of which this thread
    // takes batches half, half + kForceTPP, ...; one 16-byte index load per
    // batch, two of this thread's batches ahead.  Loads always read an existing block
    // of the list array and the value is selected afterwards (a select between
    // pointers would become a flat load).
    const int nb = STAGED ? nb0 + npl1_ld / kPlainBatch : 0;
    const uint4 zero4 = make_uint4(kHalo | (kHalo << 16), kHalo | (kHalo << 16), kHalo | (kHalo << 16),
                                   kHalo | (kHalo << 16));
    uint4 v0 = nb > half ? t0 : zero4;
    uint4 v1 = nb > half + kForceTPP ? t1 : zero4;
    for (int b = half; b < nb; b += kForceTPP) {
      uint4 t2 = l8[boff(b + 2 * kForceTPP)];
      uint4 v2 = (b + 2 * kForceTPP < nb) ? t2 : zero4;
      int j[8] = {(int)(v0.x & 0xffff), (int)(v0.x >> 16), (int)(v0.y & 0xffff), (int)(v0.y >> 16),
                  (int)(v0.z & 0xffff), (int)(v0.z >> 16), (int)(v0.w & 0xffff), (int)(v0.w >> 16)};
      double xj[8], yj[8], zj[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) { xj[u] = hx[j[u]]; yj[u] = hy[j[u]]; zj[u] = hz[j[u]]; }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        double dx = pi.x - xj[u], dy = pi.y - yj[u], dz = pi.z - zj[u];
        const double r2 = fma(dz, dz, fma(dy, dy, dx * dx));
        add_pair<VIR>(lj_masked<MIXED>(r2, rc2, sig2, eps24), dx, dy, dz, fx, fy, fz, w);
      }
      v0 = v1;
      v1 = v2;
    }
    // partners that were not staged: global memory, exact image arithmetic;
    // eight gathers in flight, the next eight indices requested ahead.  With
    // the halo each thread takes its own sub-list; without, one thread per
    // particle takes both as one sequence.
    // the sub-lists this thread takes, read as one sequence of blocks of 4
    // (sub-list s_lo, then s_hi) so that one prefetch pipeline runs across both
    // (with the halo, threads 0 and 1 of a particle take one sub-list each)
    const bool has_og = !STAGED || half < 2;
    const int s_lo = TPP > 1 ? min(half, 1) : 0, s_hi = TPP > 1 ? s_lo : 1;
    const int nbo0 = has_og ? d.n_og[s_lo * np + i] / kOtherBatch : 0;
    const int nbo = nbo0 + (has_og && s_hi != s_lo ? d.n_og[s_hi * np + i] / kOtherBatch : 0);
    const int last_ob = d.K / kOtherBatch - 1;
    auto ooff = [&](int q) -> size_t {
      const bool first = q < nbo0;
      const int blk = min(first ? q : q - nbo0, last_ob);
      return (size_t)blk * np2 + (size_t)(first ? s_lo : s_hi) * np + i;
    };
    const uint4* __restrict__ l4 = reinterpret_cast<const uint4*>(d.nlo);
    // GB blocks of 4 per round: one for the plain global layout (fewer
    // gathers in flight leave room for more waves: KG 49 -> 48 us), two with
    // the halo's remainder pieces and with DPD (one block: 138 -> 195 us)
    constexpr int GB = (STAGED || DPD) ? 2 : 1;
    uint4 jn[GB];
#pragma unroll
    for (int k = 0; k < GB; ++k) jn[k] = l4[ooff(k)];
    {
    for (int b = 0; b < nbo; b += GB) {
      // slots, and the four image codes of a block repacked into one word
      // (fewer live registers while the gathers are in flight)
      uint32_t sl[4 * GB], cq[GB];
#pragma unroll
      for (int k = 0; k < GB; ++k) {
        const uint4 jq = jn[k];
        jn[k] = l4[ooff(b + GB + k)];
        const bool in = b + k < nbo;  // the entries of this block are the list's
        sl[4 * k] = (in ? jq.x : (uint32_t)d.n) & kSlotMask;
        sl[4 * k + 1] = (in ? jq.y : (uint32_t)d.n) & kSlotMask;
        sl[4 * k + 2] = (in ? jq.z : (uint32_t)d.n) & kSlotMask;
        sl[4 * k + 3] = (in ? jq.w : (uint32_t)d.n) & kSlotMask;
        cq[k] = (jq.x >> kSlotBits) | ((jq.y >> kSlotBits) << 8) | ((jq.z >> kSlotBits) << 16) |
                (jq.w & ~kSlotMask);
        // opaque to the optimiser, so that the codes stay one packed word
        // instead of being unpacked from the entries ahead of their use
        asm("" : "+v"(cq[k]));
      }
      double4 pj[4 * GB];
#pragma unroll
      for (int u = 0; u < 4 * GB; ++u) pj[u] = P[sl[u]];
      // DPD: the partners' velocities and tags, one 32-byte gather each
      double4 vj[DPD ? 4 * GB : 1];
      if (DPD) {
#pragma unroll
        for (int u = 0; u < 4 * GB; ++u) vj[u] = VT[sl[u]];
        // every gather of the round issued before the first use (without this
        // fence the scheduler sinks each to its use, one wait per gather)
        __builtin_amdgcn_sched_barrier(0);
      }
#pragma unroll
      for (int u = 0; u < 4 * GB; ++u) {
        int sx, sy, sz;
        unpack_img((uint8_t)(cq[u >> 2] >> (8 * (u & 3))), sx, sy, sz);
        sx += sy * W;
        double dy = (pi.y - pj[u].y) - (double)sy * d.Ly;
        double dx = ((pi.x - pj[u].x) - (double)sy * Delta) - (double)sx * d.Lx;
        double dz = (pi.z - pj[u].z) - (double)sz * d.Lz;
        const double r2 = fma(dz, dz, fma(dy, dy, dx * dx));
        add_pair<VIR>(lj_masked<MIXED, CAP>(r2, rc2, sig2, eps24, d.force_cap), dx, dy, dz, fx, fy, fz, w);
        if (DPD) {
          // the image s_y boxes up streams faster by s_y gamma_dot L_y
          const double vx = (u0_ld - vj[u].x) - (double)sy * d.sv;
          dpd_pair(d, st_lo, st_hi, tag_ld, (int)vj[u].w, vx, u1_ld - vj[u].y, u2_ld - vj[u].z,
                   dx, dy, dz, r2, gx, gy, gz);
        }
      }
    }
    }
    if (BONDS && half == 0) {
      // FENE (Eq. fene), always float64; displacement by the nearest image
      int jb[2];
      double4 pb[2];
      for (int b = 0; b < 2; ++b) {
        int j = d.bond[b * np + i];
        jb[b] = j;
        if (j < 0) continue;
        double4 pj = P[j];
        pb[b] = pj;
        double dx, dy, dz;
        near_disp(d, pi, pj, Delta, dx, dy, dz);
        double r2 = dx * dx + dy * dy;
        r2 = r2 + dz * dz;
        if (!(r2 < d.fene_r02)) {
          latch(d.flags, LE_E_BOND);
          continue;
        }
        double f = -d.fene_k / (1.0 - r2 / d.fene_r02);
        add_pair<VIR>(f, dx, dy, dz, fx, fy, fz, w);
      }
      if (d.angle_k != 0.0) {
        // cosine angle term (Eq. angle): the angles centred at i (its virial
        // is counted here), at the bead below (i is its second end) and at
        // the bead above (i is its first end)
        double b1[3], b2[3], Fa[3], Fb[3];
        if (jb[0] >= 0 && jb[1] >= 0) {
          near_disp(d, pb[0], pi, Delta, b1[0], b1[1], b1[2]);
          near_disp(d, pb[1], pi, Delta, b2[0], b2[1], b2[2]);
          angle_cos(b1, b2, d.angle_k, Fa, Fb);
          fx -= Fa[0] + Fb[0]; fy -= Fa[1] + Fb[1]; fz -= Fa[2] + Fb[2];
          if (VIR) {
            // w holds twice the virial (pairs and bonds are met from both
            // ends), so the angle's single contribution enters doubled
            w[0] += 2.0 * (b1[0] * Fa[0] + b2[0] * Fb[0]);
            w[1] += 2.0 * (b1[1] * Fa[1] + b2[1] * Fb[1]);
            w[2] += 2.0 * (b1[2] * Fa[2] + b2[2] * Fb[2]);
            w[3] += 2.0 * (b1[0] * Fa[1] + b2[0] * Fb[1]);
            w[4] += 2.0 * (b1[0] * Fa[2] + b2[0] * Fb[2]);
            w[5] += 2.0 * (b1[1] * Fa[2] + b2[1] * Fb[2]);
          }
        }
        for (int b = 0; b < 2; ++b) {
          const int j = jb[b];
          if (j < 0) continue;
          const int j2 = d.bond[b * np + j];  // the next bead beyond j
          if (j2 < 0) continue;
          const double4 p2 = P[j2];
          // angle (j2, j, i) below or (i, j, j2) above; i's force is that of its end
          near_disp(d, p2, pb[b], Delta, b1[0], b1[1], b1[2]);
          near_disp(d, pi, pb[b], Delta, b2[0], b2[1], b2[2]);
          angle_cos(b1, b2, d.angle_k, Fa, Fb);
          fx += Fb[0]; fy += Fb[1]; fz += Fb[2];
        }
      }
    }
  }
  if (STAGED) {
    // the other threads of each particle hand over their partial sums (the
    // halo array is free once every thread has left the pair loops); the
    // first adds them in thread order
    __syncthreads();
    if (half > 0) {
      double* ex = hbuf + ((half - 1) * kTile + tl) * 9;
      ex[0] = fx; ex[1] = fy; ex[2] = fz;
      if (VIR) for (int q = 0; q < 6; ++q) ex[3 + q] = w[q];
    }
    __syncthreads();
    if (half == 0) {
      for (int t = 1; t < kForceTPP; ++t) {
        const double* ex = hbuf + ((t - 1) * kTile + tl) * 9;
        fx += ex[0]; fy += ex[1]; fz += ex[2];
        if (VIR) for (int q = 0; q < 6; ++q) w[q] += ex[3 + q];
      }
    } else {
      for (int q = 0; q < 6; ++q) w[q] = 0.0;
    }
  }
  if constexpr (!STAGED && TPP > 1) {
    // the thread of sub-list 1 hands its sums (pair forces, virial, DPD terms)
    // to the thread of sub-list 0, which adds them after its own
    constexpr int XW = DPD ? 12 : 9;
    __shared__ double xch[kTile * XW];
    if (half == 1) {
      double* ex = xch + tl * XW;
      ex[0] = fx; ex[1] = fy; ex[2] = fz;
      if (VIR) for (int q = 0; q < 6; ++q) ex[3 + q] = w[q];
      if (DPD) { ex[9] = gx; ex[10] = gy; ex[11] = gz; }
    }
    __syncthreads();
    if (half == 0) {
      const double* ex = xch + tl * XW;
      fx += ex[0]; fy += ex[1]; fz += ex[2];
      if (VIR) for (int q = 0; q < 6; ++q) w[q] += ex[3 + q];
      if (DPD) { gx += ex[9]; gy += ex[10]; gz += ex[11]; }
    } else {
      for (int q = 0; q < 6; ++q) w[q] = 0.0;
    }
  }
  const bool ep = valid && half == 0;  // threads that finish a particle
  double kin[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  double v2 = 0.0;
  if (MODE == kForcesOnly) {
    if (ep) {
      int t = tag_ld;
      if (f_out) {
        f_out[t] = fx; f_out[d.n + t] = fy; f_out[2 * d.n + t] = fz;
      }
      double cx = u0_ld - d.c_sr * (pi.y - 0.5 * d.Ly);
      double cy = u1_ld, cz = u2_ld;
      double m = d.mass;
      kin[0] = m * cx * cx; kin[1] = m * cy * cy; kin[2] = m * cz * cz;
      kin[3] = m * cx * cy; kin[4] = m * cx * cz; kin[5] = m * cy * cz;
    }
  } else if (DPD) {
    if (ep) {
      double* F = d.frc[ac];
      F[i] = fx + gx; F[np + i] = fy + gy; F[2 * np + i] = fz + gz;
    }
  } else if (ep) {
    double* U = d.vel[ac];
    double ux = u0_ld, uy = u1_ld, uz = u2_ld;
    int t = tag_ld;
    uint32_t ctr[4] = {st_lo, st_hi, (uint32_t)t, 0u};
    philox(ctr, d.seed_lo, d.seed_hi);
    // friction velocity: peculiar (Eq. vi), or the lab velocity of the image
    // inside the box (positions are wrapped lazily, so a particle above the
    // top face still carries the velocity it had before crossing)
    double cx = d.thermostat == LE_THERMO_LANGEVIN_LAB ? ux - d.sv * floor(pi.y / d.Ly)
                                                       : ux - d.c_sr * (pi.y - 0.5 * d.Ly);
    double Fx = (fx - d.gamma_m * cx) + d.pref * u01c(ctr[0]);
    double Fy = (fy - d.gamma_m * uy) + d.pref * u01c(ctr[1]);
    double Fz = (fz - d.gamma_m * uz) + d.pref * u01c(ctr[2]);
    if (MODE == kInitForce) {
      double* F = d.frc[ac];
      F[i] = Fx; F[np + i] = Fy; F[2 * np + i] = Fz;
    } else {
      ux = ux + d.h * Fx; uy = uy + d.h * Fy; uz = uz + d.h * Fz;
      if (SAMPLE) {
        double m = d.mass;
        double cxn = ux - d.c_sr * (pi.y - 0.5 * d.Ly);
        kin[0] = m * cxn * cxn; kin[1] = m * uy * uy; kin[2] = m * uz * uz;
        kin[3] = m * cxn * uy; kin[4] = m * cxn * uz; kin[5] = m * uy * uz;
      }
      if (MODE == kStepLast) {
        double* F = d.frc[ac];
        F[i] = Fx; F[np + i] = Fy; F[2 * np + i] = Fz;
      } else {
        ux = ux + d.h * Fx; uy = uy + d.h * Fy; uz = uz + d.h * Fz;
        double cxh = ux - d.c_sr * (pi.y - 0.5 * d.Ly);
        v2 = cxh * cxh + uy * uy + uz * uz;
        double4 q;
        q.x = pi.x + d.dt * (ux + d.drift_sr * (pi.y - 0.5 * d.Ly));
        q.y = pi.y + d.dt * uy;
        q.z = pi.z + d.dt * uz;
        q.w = pi.w;
        reinterpret_cast<double4*>(d.pos[1 - pc])[i] = q;
        if (!(isfinite(q.x) && isfinite(q.y) && isfinite(q.z))) latch(d.flags, LE_E_NONFINITE);
      }
      U[i] = ux; U[np + i] = uy; U[2 * np + i] = uz;
    }
  }
  if (MODE == kStepFused) vmax_commit<kTh>(d, v2, lb);
  if (VIR) {
    double vals[kStressComps];
#pragma unroll
    for (int k = 0; k < 6; ++k) { vals[k] = kin[k]; vals[6 + k] = 0.5 * w[k]; }
    block_partials<kTh>(vals, d.partials, lb);
  }
}

template <int MODE, bool MIXED, bool BONDS, bool SAMPLE, bool STAGED, bool CAP = false>
__global__ void __launch_bounds__(STAGED ? kForceTPP * kTile : 4 * kTile)
    k_force(Dev d, double* __restrict__ f_out, double* __restrict__ sample_out) {
  (void)sample_out;
  force_body<MODE, MIXED, BONDS, SAMPLE, STAGED, CAP>(d, xcd_block(d.ntiles), f_out);
}

// Batched form (the step modes; no per-particle output): one launch over the
// tiles of every simulation of the batch.  Global layout: XCD-remapped over
// the whole grid (partner gathers hit the L2 of the XCD that holds the
// region); LDS halo: runs of 16 tiles dealt round-robin to the XCDs, which
// evens out members of unequal cost per tile (64-request batch 0.711 ->
// 0.699 ms per step; the KG melts of the global layout gain nothing from it).
// Plain DPD steps (global layout, no stress sample): held to 168 VGPRs, three
// waves per SIMD instead of two, which the kernel reaches without spills (the
// sampling variant would spill, so it keeps the plain bound).
template <bool MIXED, bool BONDS>
__global__ void __launch_bounds__(4 * kTile) __attribute__((amdgpu_waves_per_eu(3)))
    k_force_dpd(Dev d, double* __restrict__ f_out, double* __restrict__ sample_out) {
  (void)sample_out;
  force_body<kDpdForce, MIXED, BONDS, false, false, false>(d, xcd_block(d.ntiles), f_out);
}
template <int MODE, bool MIXED, bool BONDS, bool SAMPLE, bool STAGED, bool CAP = false>
__global__ void __launch_bounds__(STAGED ? kForceTPP * kTile : 4 * kTile) k_force_b(Batch b) {
  int sm, lb;
  const int g = STAGED ? xcd_spread<16>((int)blockIdx.x, (int)gridDim.x) : xcd_map((int)blockIdx.x, (int)gridDim.x);
  locate(b, g, sm, lb);
  force_body<MODE, MIXED, BONDS, SAMPLE, STAGED, CAP>(stage_dev(b.dev[sm]), lb, nullptr);
}

// DPD: pack the current velocities and tags of every slot (and zeros for the
// sentinel slot n) into vt, so that the force kernel gathers one 32-byte
// record per partner.
__device__ __forceinline__ void pack_vt_body(const Dev& d, int bid) {
  if (d.flags->status) return;
  const Ctrl* c = d.ctrl;
  const int i = bid * kBlock + threadIdx.x;
  const int np = d.np;
  double4 v = make_double4(0.0, 0.0, 0.0, 0.0);
  if (i < d.n) {
    const double* U = d.vel[c->aux_cur];
    v = make_double4(U[i], U[np + i], U[2 * np + i], (double)d.tag[c->aux_cur][i]);
  }
  if (i <= d.n) reinterpret_cast<double4*>(d.vt)[i] = v;
}

__global__ void __launch_bounds__(kBlock) k_pack_vt(Dev d) { pack_vt_body(d, blockIdx.x); }

__global__ void __launch_bounds__(kBlock) k_pack_vt_b(Batch b) {
  int sm, bid;
  locate(b, blockIdx.x, sm, bid);
  pack_vt_body(stage_dev(b.dev[sm]), bid);
}

// DPD steps, after k_force<kDpdForce>: u += dt/(2m) F (the step's second
// half-kick); with SAMPLE the kinetic stress partials of the new full-step
// velocities go to partials[block][0..5] (the force kernel wrote the virial
// to [6..11]); unless LAST, the next half-kick and drift follow as in the
// fused Langevin step.  One thread per slot, blocks of kTile.
template <bool LAST, bool SAMPLE>
__device__ __forceinline__ void integrate_body(const Dev& d, int bid) {
  __shared__ int skip;
  Ctrl* c = d.ctrl;
  if (threadIdx.x == 0) skip = d.flags->status;
  __syncthreads();
  if (skip) return;
  const int i = bid * kTile + threadIdx.x;
  const int np = d.np;
  double kin[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  double v2 = 0.0;
  if (i < d.n) {
    const int pc = c->pos_cur, ac = c->aux_cur;
    const double4 p = reinterpret_cast<const double4*>(d.pos[pc])[i];
    double* U = d.vel[ac];
    const double* F = d.frc[ac];
    const double Fx = F[i], Fy = F[np + i], Fz = F[2 * np + i];
    double ux = U[i] + d.h * Fx;
    double uy = U[np + i] + d.h * Fy;
    double uz = U[2 * np + i] + d.h * Fz;
    if (SAMPLE) {
      const double m = d.mass;
      const double cx = ux - d.c_sr * (p.y - 0.5 * d.Ly);
      kin[0] = m * cx * cx; kin[1] = m * uy * uy; kin[2] = m * uz * uz;
      kin[3] = m * cx * uy; kin[4] = m * cx * uz; kin[5] = m * uy * uz;
    }
    if (!LAST) {
      ux = ux + d.h * Fx; uy = uy + d.h * Fy; uz = uz + d.h * Fz;
      const double cxh = ux - d.c_sr * (p.y - 0.5 * d.Ly);
      v2 = cxh * cxh + uy * uy + uz * uz;
      double4 q;
      q.x = p.x + d.dt * (ux + d.drift_sr * (p.y - 0.5 * d.Ly));
      q.y = p.y + d.dt * uy;
      q.z = p.z + d.dt * uz;
      q.w = p.w;
      reinterpret_cast<double4*>(d.pos[1 - pc])[i] = q;
      if (!(isfinite(q.x) && isfinite(q.y) && isfinite(q.z))) latch(d.flags, LE_E_NONFINITE);
    }
    U[i] = ux; U[np + i] = uy; U[2 * np + i] = uz;
  }
  if (!LAST) vmax_commit<kTile>(d, v2, bid);
  if (SAMPLE) {
    double vals[kStressComps];
#pragma unroll
    for (int k = 0; k < 6; ++k) { vals[k] = kin[k]; vals[6 + k] = 0.0; }
    block_partials<kTile>(vals, d.partials, bid, 6);
  }
}

template <bool LAST, bool SAMPLE>
__global__ void __launch_bounds__(kTile) k_integrate(Dev d) { integrate_body<LAST, SAMPLE>(d, blockIdx.x); }

template <bool LAST, bool SAMPLE>
__global__ void __launch_bounds__(kTile) k_integrate_b(Batch b) {
  int sm, bid;
  locate(b, blockIdx.x, sm, bid);
  integrate_body<LAST, SAMPLE>(stage_dev(b.dev[sm]), bid);
}

// Stand-alone reduction of the block partials (le_forces, le_stress).
__global__ void k_stress_final(Dev d, double* out6, int virial_only) {
  __shared__ int skip;
  if (threadIdx.x == 0) skip = d.flags->status;
  __syncthreads();
  if (skip) return;
  reduce_partials(d, out6, virial_only != 0);
}

// Batched form: block k reduces simulation k's partials into out.ptr[k].
__global__ void k_stress_final_b(Batch b, BatchOut out) {
  const Dev& d = stage_dev(b.dev[blockIdx.x]);
  __shared__ int skip;
  if (threadIdx.x == 0) skip = d.flags->status;
  __syncthreads();
  if (skip) return;
  reduce_partials(d, out.ptr[blockIdx.x], false);
}

// Copy the current control state and speed-bound words into the other copy
// (a no-op for the simulation; lets a captured graph start on its copy).
__global__ void k_ctrl_copy(const Ctrl* __restrict__ src, Ctrl* __restrict__ dst,
                            const unsigned long long* __restrict__ vsrc,
                            unsigned long long* __restrict__ vdst) {
  if (threadIdx.x == 0) *dst = *src;
  for (int k = threadIdx.x; k < kSlots * kLineU64; k += blockDim.x) vdst[k] = vsrc[k];
}

// ---------------------------------------------------------- observables
// Per block: bin of each particle (its image in the box, with the matching
// lab u_x), then one thread per bin sums the block's particles of that bin in
// index order; kinetic and centre-of-mass sums by wave shuffles.  The final
// kernel adds the block partials in block order.
constexpr int kObsStride = 3 * LE_MAX_BINS + 4;

__global__ void __launch_bounds__(kBlock) k_obs_partial(Dev d, int nbins) {
  __shared__ int sbin[kBlock];
  __shared__ double sux[kBlock], smc[kBlock];
  __shared__ double red[kBlock / 64][4];
  if (d.flags->status) return;
  const Ctrl* c = d.ctrl;
  const int i = blockIdx.x * kBlock + threadIdx.x;
  const int np = d.np;
  int b = -1;
  double ux = 0.0, mc2 = 0.0, v[4] = {0.0, 0.0, 0.0, 0.0};
  if (i < d.n) {
    const double4 p = reinterpret_cast<const double4*>(d.pos[c->pos_cur])[i];
    const double* U = d.vel[c->aux_cur];
    const double u0 = U[i], u1 = U[np + i], u2 = U[2 * np + i];
    double y = p.y;
    const double ky = wrap1(y, d.Ly);
    ux = (u0 - ky * d.jump_sv) + d.drift_sr * (y - 0.5 * d.Ly);  // lab u_x of the in-box image
    b = (int)(y / d.Ly * (double)nbins);
    if (b < 0) b = 0;
    if (b > nbins - 1) b = nbins - 1;
    const double cx = u0 - d.c_sr * (p.y - 0.5 * d.Ly);
    mc2 = d.mass * (cx * cx + u1 * u1 + u2 * u2);
    v[0] = mc2;
    v[1] = ux; v[2] = u1; v[3] = u2;
  }
  sbin[threadIdx.x] = b;
  sux[threadIdx.x] = ux;
  smc[threadIdx.x] = mc2;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    double t = v[k];
    for (int o = 32; o > 0; o >>= 1) t += __shfl_xor(t, o, 64);
    if (lane == 0) red[wid][k] = t;
  }
  __syncthreads();
  double* out = d.obs_part + (size_t)blockIdx.x * kObsStride;
  for (int bb = threadIdx.x; bb < nbins; bb += kBlock) {
    double cnt = 0.0, sum = 0.0, sk = 0.0;
    for (int q = 0; q < kBlock; ++q)
      if (sbin[q] == bb) { cnt += 1.0; sum += sux[q]; sk += smc[q]; }
    out[bb] = cnt;
    out[nbins + bb] = sum;
    out[2 * nbins + bb] = sk;
  }
  if (threadIdx.x < 4) {
    double t = 0.0;
    for (int w = 0; w < kBlock / 64; ++w) t += red[w][threadIdx.x];
    out[3 * nbins + threadIdx.x] = t;
  }
}

__global__ void __launch_bounds__(kBlock) k_obs_final(Dev d, int nbins, int nblk, double* out) {
  if (d.flags->status) return;
  for (int k = threadIdx.x; k < 3 * nbins + 4; k += kBlock) {
    double t = 0.0;
    for (int b = 0; b < nblk; ++b) t += d.obs_part[(size_t)b * kObsStride + k];
    if (k == 3 * nbins) t = t / (3.0 * (double)d.n - 3.0);
    else if (k > 3 * nbins) t = t / (double)d.n;
    out[k] = t;
  }
}

// Unwrapped y, z of every particle (slot order in, tag order out).
__global__ void __launch_bounds__(kBlock) k_unwrapped(Dev d, double* __restrict__ out) {
  if (d.flags->status) return;
  const Ctrl* c = d.ctrl;
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= d.n) return;
  const double4 p = reinterpret_cast<const double4*>(d.pos[c->pos_cur])[i];
  int ky, kz;
  img_get(p.w, ky, kz);
  const int t = d.tag[c->aux_cur][i];
  out[t] = p.y + (double)ky * d.Ly;
  out[d.n + t] = p.z + (double)kz * d.Lz;
}

// Mean squared y, z displacement against ref (tag order): block partials in
// obs_part, then one block sums them in block order.
__global__ void __launch_bounds__(kBlock) k_msd_partial(Dev d, const double* __restrict__ ref) {
  __shared__ double red[kBlock / 64][2];
  if (d.flags->status) return;
  const Ctrl* c = d.ctrl;
  const int i = blockIdx.x * kBlock + threadIdx.x;
  double v[2] = {0.0, 0.0};
  if (i < d.n) {
    const double4 p = reinterpret_cast<const double4*>(d.pos[c->pos_cur])[i];
    int ky, kz;
    img_get(p.w, ky, kz);
    const int t = d.tag[c->aux_cur][i];
    const double dy = (p.y + (double)ky * d.Ly) - ref[t];
    const double dz = (p.z + (double)kz * d.Lz) - ref[d.n + t];
    v[0] = dy * dy;
    v[1] = dz * dz;
  }
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  for (int k = 0; k < 2; ++k) {
    double t = v[k];
    for (int o = 32; o > 0; o >>= 1) t += __shfl_xor(t, o, 64);
    if (lane == 0) red[wid][k] = t;
  }
  __syncthreads();
  if (threadIdx.x < 2) {
    double t = 0.0;
    for (int w = 0; w < kBlock / 64; ++w) t += red[w][threadIdx.x];
    d.obs_part[(size_t)blockIdx.x * kObsStride + threadIdx.x] = t;
  }
}

__global__ void __launch_bounds__(kBlock) k_msd_final(Dev d, int nblk, double* out2) {
  __shared__ double red[kBlock / 64][2];
  if (d.flags->status) return;
  double v[2] = {0.0, 0.0};
  for (int b = threadIdx.x; b < nblk; b += kBlock) {
    v[0] += d.obs_part[(size_t)b * kObsStride];
    v[1] += d.obs_part[(size_t)b * kObsStride + 1];
  }
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  for (int k = 0; k < 2; ++k) {
    double t = v[k];
    for (int o = 32; o > 0; o >>= 1) t += __shfl_xor(t, o, 64);
    if (lane == 0) red[wid][k] = t;
  }
  __syncthreads();
  if (threadIdx.x < 2) {
    double t = 0.0;
    for (int w = 0; w < kBlock / 64; ++w) t += red[w][threadIdx.x];
    out2[threadIdx.x] = t / (double)d.n;
  }
}

// ----------------------------------------------------------- state out
__global__ void k_state_out(Dev d, double* x, double* u, int32_t* cell_of, int32_t* order) {
  if (d.flags->status) return;
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= d.n) return;
  const Ctrl* c = d.ctrl;
  const int np = d.np, n = d.n;
  const int ac = c->aux_cur;
  int t = d.tag[ac][i];
  double4 p = reinterpret_cast<const double4*>(d.pos[c->pos_cur])[i];
  if (x) { x[t] = p.x; x[n + t] = p.y; x[2 * n + t] = p.z; }
  if (u) for (int a = 0; a < 3; ++a) u[a * n + t] = d.vel[ac][a * np + i];
  if (cell_of) {
    int ix = cell_index(p.x, d.inv_lx, d.nx);
    int iy = cell_index(p.y, d.inv_ly, d.ny);
    int iz = cell_index(p.z, d.inv_lz, d.nz);
    cell_of[t] = (iz * d.ny + iy) * d.nx + ix;
  }
  if (order) order[i] = t;
}

__global__ void k_pairs_out(Dev d, int64_t* pairs, int64_t cap, unsigned long long* counter) {
  if (d.flags->status) return;
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= d.n) return;
  const int np = d.np;
  const int32_t* tag = d.tag[d.ctrl->aux_cur];
  const int* hs = d.halo_slot + (size_t)(i / kTile) * kHalo;
  const int ti = tag[i];
  const int np2 = d.np2;
  for (int sub = 0; sub < 2; ++sub) {
  const int v = sub * np + i;
  const int npl = d.n_plain[v], nog = d.n_og[v];
  for (int k = 0; k < npl + nog; ++k) {
    int slot;
    if (k < npl) {
      int h = d.nl16[idx8(k, v, np2)];
      if (h == kHalo) continue;
      slot = hs[h];
    } else {
      slot = (int)(d.nlo[idx4(k - npl, v, np2)] & kSlotMask);
      if (slot == d.n) continue;
    }
    int tj = tag[slot];
    if (ti < tj) {
      unsigned long long idx = atomicAdd(counter, 1ull);
      if ((int64_t)idx < cap) { pairs[2 * idx] = ti; pairs[2 * idx + 1] = tj; }
    }
  }
  }
}

// Copy the latched status word to a caller's device int32 (stream-ordered).
__global__ void k_status_out(const Flags* __restrict__ f, int32_t* __restrict__ out) {
  if (threadIdx.x == 0) *out = f->status;
}

// ------------------------------------------------------------- test hooks
__global__ void k_offsets(double sv, double Lx, double dt, int64_t step0, int64_t count, double* out) {
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < count) out[k] = le_offset(step0 + k, dt, sv, Lx);
}

__global__ void k_philox(const uint32_t* ctr, const uint32_t* key, uint32_t* out, int64_t count) {
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= count) return;
  uint32_t c[4] = {ctr[4 * k], ctr[4 * k + 1], ctr[4 * k + 2], ctr[4 * k + 3]};
  philox(c, key[2 * k], key[2 * k + 1]);
  for (int a = 0; a < 4; ++a) out[4 * k + a] = c[a];
}

// ---------------------------------------------------------------- launchers
static inline int blocks_for(int64_t n) { return (int)((n + kBlock - 1) / kBlock); }

hipError_t launch_load_state(const Dev& d, hipStream_t s, const double* x0, const double* u0,
                             const double* f0, int64_t step0, double Delta0) {
  int nb = blocks_for(d.n > d.ncell ? d.n : d.ncell);
  hipLaunchKernelGGL(k_load_state, dim3(nb), dim3(kBlock), 0, s, d, x0, u0, f0, step0, Delta0);
  return hipGetLastError();
}

hipError_t launch_rebuild(const Dev& d, Ctrl* next, unsigned long long* next_vmax, hipStream_t s,
                          bool force, bool control) {
  // kernels after the first see the control copy it writes
  Dev dn = d;
  dn.ctrl = next;
  dn.vmax = next_vmax;
  hipLaunchKernelGGL(k_control_bin, dim3((d.n + kBinBlock - 1) / kBinBlock), dim3(kBlock), 0, s, d, next, next_vmax,
                     force ? 1 : 0, control ? 1 : 0);
  hipLaunchKernelGGL(k_scan_permute, dim3(d.sp_blocks), dim3(kBlock), 0, s, dn);
  // the LDS halo of the search: full size, or smaller (more blocks per CU)
  // for sparse systems whose lists hold global slots
  if (dn.staged) hipLaunchKernelGGL((k_neighbors<kHalo, false>), dim3(d.ntiles), dim3(2 * kTile), 0, s, dn);
  else if (dn.small_halo)
    hipLaunchKernelGGL((k_neighbors<kHaloSearch, true>), dim3(d.ntiles), dim3(2 * kTile), 0, s, dn);
  else hipLaunchKernelGGL((k_neighbors<kHalo, true>), dim3(d.ntiles), dim3(2 * kTile), 0, s, dn);
  return hipGetLastError();
}
hipError_t launch_kick_drift(const Dev& d, hipStream_t s) {
  hipLaunchKernelGGL(k_kick_drift, dim3(blocks_for(d.n)), dim3(kBlock), 0, s, d);
  return hipGetLastError();
}

// The force launches go through hipExtLaunchKernelGGL so that optional
// events (e0, e1) take the timestamps of the dispatch itself.
template <typename K>
static void launch_k(K k, dim3 g, dim3 b, hipStream_t s, hipEvent_t e0, hipEvent_t e1, const Dev& d,
                     double* f_out, double* so) {
  if (e0 || e1) hipExtLaunchKernelGGL(k, g, b, 0, s, e0, e1, 0, d, f_out, so);
  else hipLaunchKernelGGL(k, g, b, 0, s, d, f_out, so);
}
template <int MODE, bool SAMPLE, bool STAGED>
static void launch_force_s(const Dev& d, hipStream_t s, double* f_out, double* so, hipEvent_t e0,
                           hipEvent_t e1) {
  dim3 g(d.ntiles), b(STAGED ? kForceTPP * kTile : kGlobalTPP * kTile);
  const bool bonds = d.chain_len > 0;
  const bool mixed = d.precision == LE_MIXED;
  if constexpr (!STAGED && MODE != kDpdForce) {
    if (d.force_cap > 0.0) {  // the host guarantees FP64 and the global layout
      if (bonds) launch_k(k_force<MODE, false, true, SAMPLE, false, true>, g, b, s, e0, e1, d, f_out, so);
      else launch_k(k_force<MODE, false, false, SAMPLE, false, true>, g, b, s, e0, e1, d, f_out, so);
      return;
    }
  }
  if constexpr (MODE == kDpdForce && !SAMPLE && !STAGED) {
    if (mixed) {
      if (bonds) launch_k(k_force_dpd<true, true>, g, b, s, e0, e1, d, f_out, so);
      else launch_k(k_force_dpd<true, false>, g, b, s, e0, e1, d, f_out, so);
    } else {
      if (bonds) launch_k(k_force_dpd<false, true>, g, b, s, e0, e1, d, f_out, so);
      else launch_k(k_force_dpd<false, false>, g, b, s, e0, e1, d, f_out, so);
    }
  } else if (mixed) {
    if (bonds) launch_k(k_force<MODE, true, true, SAMPLE, STAGED>, g, b, s, e0, e1, d, f_out, so);
    else launch_k(k_force<MODE, true, false, SAMPLE, STAGED>, g, b, s, e0, e1, d, f_out, so);
  } else {
    if (bonds) launch_k(k_force<MODE, false, true, SAMPLE, STAGED>, g, b, s, e0, e1, d, f_out, so);
    else launch_k(k_force<MODE, false, false, SAMPLE, STAGED>, g, b, s, e0, e1, d, f_out, so);
  }
}
template <int MODE, bool SAMPLE>
static void launch_force_t(const Dev& d, hipStream_t s, double* f_out, double* so, hipEvent_t e0,
                           hipEvent_t e1) {
  if (d.staged) launch_force_s<MODE, SAMPLE, true>(d, s, f_out, so, e0, e1);
  else launch_force_s<MODE, SAMPLE, false>(d, s, f_out, so, e0, e1);
}

hipError_t launch_force(const Dev& d, hipStream_t s, ForceMode mode, bool sample, double* f_out,
                        double* sample_out, hipEvent_t e0, hipEvent_t e1) {
  switch (mode) {
    case kForcesOnly: launch_force_t<kForcesOnly, false>(d, s, f_out, nullptr, e0, e1); break;
    case kInitForce: launch_force_t<kInitForce, false>(d, s, f_out, nullptr, e0, e1); break;
    case kStepLast:
      if (sample) launch_force_t<kStepLast, true>(d, s, f_out, sample_out, e0, e1);
      else launch_force_t<kStepLast, false>(d, s, f_out, nullptr, e0, e1);
      break;
    case kStepFused:
      if (sample) launch_force_t<kStepFused, true>(d, s, f_out, sample_out, e0, e1);
      else launch_force_t<kStepFused, false>(d, s, f_out, nullptr, e0, e1);
      break;
    case kDpdForce:
      if (d.staged || !d.vt) return hipErrorInvalidValue;  // DPD partners come from global memory
      hipLaunchKernelGGL(k_pack_vt, dim3(blocks_for(d.n + 1)), dim3(kBlock), 0, s, d);
      if (sample) launch_force_s<kDpdForce, true, false>(d, s, f_out, sample_out, e0, e1);
      else launch_force_s<kDpdForce, false, false>(d, s, f_out, nullptr, e0, e1);
      break;
  }
  return hipGetLastError();
}

hipError_t launch_integrate(const Dev& d, hipStream_t s, bool last, bool sample) {
  dim3 g(d.ntiles), b(kTile);
  if (last) {
    if (sample) hipLaunchKernelGGL((k_integrate<true, true>), g, b, 0, s, d);
    else hipLaunchKernelGGL((k_integrate<true, false>), g, b, 0, s, d);
  } else {
    if (sample) hipLaunchKernelGGL((k_integrate<false, true>), g, b, 0, s, d);
    else hipLaunchKernelGGL((k_integrate<false, false>), g, b, 0, s, d);
  }
  return hipGetLastError();
}

hipError_t launch_stress_final(const Dev& d, hipStream_t s, double* out6, bool virial_only) {
  hipLaunchKernelGGL(k_stress_final, dim3(1), dim3(kBlock), 0, s, d, out6, virial_only ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_ctrl_copy(const Ctrl* src, Ctrl* dst, const unsigned long long* vsrc,
                            unsigned long long* vdst, hipStream_t s) {
  hipLaunchKernelGGL(k_ctrl_copy, dim3(1), dim3(64), 0, s, src, dst, vsrc, vdst);
  return hipGetLastError();
}
hipError_t launch_observables(const Dev& d, hipStream_t s, int nbins, double* out) {
  const int nblk = blocks_for(d.n);
  hipLaunchKernelGGL(k_obs_partial, dim3(nblk), dim3(kBlock), 0, s, d, nbins);
  hipLaunchKernelGGL(k_obs_final, dim3(1), dim3(kBlock), 0, s, d, nbins, nblk, out);
  return hipGetLastError();
}
hipError_t launch_unwrapped(const Dev& d, hipStream_t s, double* out) {
  hipLaunchKernelGGL(k_unwrapped, dim3(blocks_for(d.n)), dim3(kBlock), 0, s, d, out);
  return hipGetLastError();
}
hipError_t launch_msd(const Dev& d, hipStream_t s, const double* ref, double* out2) {
  const int nblk = blocks_for(d.n);
  hipLaunchKernelGGL(k_msd_partial, dim3(nblk), dim3(kBlock), 0, s, d, ref);
  hipLaunchKernelGGL(k_msd_final, dim3(1), dim3(kBlock), 0, s, d, nblk, out2);
  return hipGetLastError();
}
hipError_t launch_state_out(const Dev& d, hipStream_t s, double* x, double* u, int32_t* cell_of,
                            int32_t* order) {
  hipLaunchKernelGGL(k_state_out, dim3(blocks_for(d.n)), dim3(kBlock), 0, s, d, x, u, cell_of, order);
  return hipGetLastError();
}

hipError_t launch_pairs_out(const Dev& d, hipStream_t s, int64_t* pairs, int64_t cap,
                            unsigned long long* counter) {
  hipLaunchKernelGGL(k_pairs_out, dim3(blocks_for(d.n)), dim3(kBlock), 0, s, d, pairs, cap, counter);
  return hipGetLastError();
}

// ------------------------------------------------------- batched launchers
__global__ void k_store_dev(Dev a, Dev b, Dev* dst) {
  if (threadIdx.x == 0) {
    dst[0] = a;
    dst[1] = b;
  }
}

hipError_t launch_store_dev(const Dev& a, const Dev& b, Dev* dst, hipStream_t s) {
  hipLaunchKernelGGL(k_store_dev, dim3(1), dim3(64), 0, s, a, b, dst);
  return hipGetLastError();
}

static inline dim3 grid_of(const Batch& b) { return dim3((unsigned)b.start[b.nsims]); }

hipError_t launch_kick_drift_b(const Batch& par_cur, hipStream_t s) {
  hipLaunchKernelGGL(k_kick_drift_b, grid_of(par_cur), dim3(kBlock), 0, s, par_cur);
  return hipGetLastError();
}

hipError_t launch_rebuild_b(const Batch& bin_cur, const Batch& scan_nxt, const Batch& tile_nxt,
                            const Dev& cfg, hipStream_t s) {
  hipLaunchKernelGGL(k_control_bin_b, grid_of(bin_cur), dim3(kBlock), 0, s, bin_cur);
  hipLaunchKernelGGL(k_scan_permute_b, grid_of(scan_nxt), dim3(kBlock), 0, s, scan_nxt);
  if (cfg.staged) hipLaunchKernelGGL((k_neighbors_b<kHalo, false>), grid_of(tile_nxt), dim3(2 * kTile), 0, s, tile_nxt);
  else if (cfg.small_halo)
    hipLaunchKernelGGL((k_neighbors_b<kHaloSearch, true>), grid_of(tile_nxt), dim3(2 * kTile), 0, s, tile_nxt);
  else hipLaunchKernelGGL((k_neighbors_b<kHalo, true>), grid_of(tile_nxt), dim3(2 * kTile), 0, s, tile_nxt);
  return hipGetLastError();
}

template <int MODE, bool SAMPLE, bool STAGED>
static void launch_force_bs(const Batch& b, const Dev& cfg, hipStream_t s) {
  const dim3 g = grid_of(b), blk(STAGED ? kForceTPP * kTile : kGlobalTPP * kTile);
  const bool bonds = cfg.chain_len > 0;
  if constexpr (!STAGED && MODE != kDpdForce) {
    if (cfg.force_cap > 0.0) {
      if (bonds) hipLaunchKernelGGL((k_force_b<MODE, false, true, SAMPLE, false, true>), g, blk, 0, s, b);
      else hipLaunchKernelGGL((k_force_b<MODE, false, false, SAMPLE, false, true>), g, blk, 0, s, b);
      return;
    }
  }
  if (cfg.precision == LE_MIXED) {
    if (bonds) hipLaunchKernelGGL((k_force_b<MODE, true, true, SAMPLE, STAGED>), g, blk, 0, s, b);
    else hipLaunchKernelGGL((k_force_b<MODE, true, false, SAMPLE, STAGED>), g, blk, 0, s, b);
  } else {
    if (bonds) hipLaunchKernelGGL((k_force_b<MODE, false, true, SAMPLE, STAGED>), g, blk, 0, s, b);
    else hipLaunchKernelGGL((k_force_b<MODE, false, false, SAMPLE, STAGED>), g, blk, 0, s, b);
  }
}

template <int MODE, bool SAMPLE>
static void launch_force_bt(const Batch& b, const Dev& cfg, hipStream_t s) {
  if (cfg.staged) launch_force_bs<MODE, SAMPLE, true>(b, cfg, s);
  else launch_force_bs<MODE, SAMPLE, false>(b, cfg, s);
}

hipError_t launch_force_b(const Batch& tile_cur, const Batch& par_cur, const Dev& cfg, hipStream_t s,
                          ForceMode mode, bool sample) {
  switch (mode) {
    case kStepLast:
      if (sample) launch_force_bt<kStepLast, true>(tile_cur, cfg, s);
      else launch_force_bt<kStepLast, false>(tile_cur, cfg, s);
      break;
    case kStepFused:
      if (sample) launch_force_bt<kStepFused, true>(tile_cur, cfg, s);
      else launch_force_bt<kStepFused, false>(tile_cur, cfg, s);
      break;
    case kDpdForce:
      if (cfg.staged || !cfg.vt) return hipErrorInvalidValue;
      hipLaunchKernelGGL(k_pack_vt_b, grid_of(par_cur), dim3(kBlock), 0, s, par_cur);
      if (sample) launch_force_bs<kDpdForce, true, false>(tile_cur, cfg, s);
      else launch_force_bs<kDpdForce, false, false>(tile_cur, cfg, s);
      break;
    default:
      return hipErrorInvalidValue;  // the other modes are not batched
  }
  return hipGetLastError();
}

hipError_t launch_integrate_b(const Batch& tile_cur, hipStream_t s, bool last, bool sample) {
  const dim3 g = grid_of(tile_cur), b(kTile);
  if (last) {
    if (sample) hipLaunchKernelGGL((k_integrate_b<true, true>), g, b, 0, s, tile_cur);
    else hipLaunchKernelGGL((k_integrate_b<true, false>), g, b, 0, s, tile_cur);
  } else {
    if (sample) hipLaunchKernelGGL((k_integrate_b<false, true>), g, b, 0, s, tile_cur);
    else hipLaunchKernelGGL((k_integrate_b<false, false>), g, b, 0, s, tile_cur);
  }
  return hipGetLastError();
}

hipError_t launch_stress_final_b(const Batch& one_cur, const BatchOut& out, hipStream_t s) {
  hipLaunchKernelGGL(k_stress_final_b, dim3((unsigned)one_cur.nsims), dim3(kBlock), 0, s, one_cur, out);
  return hipGetLastError();
}

hipError_t launch_status_out(const Dev& d, hipStream_t s, int32_t* out) {
  hipLaunchKernelGGL(k_status_out, dim3(1), dim3(64), 0, s, d.flags, out);
  return hipGetLastError();
}

hipError_t launch_offsets(double sr, double Lx, double Ly, double dt, int64_t step0, int64_t count,
                          double* out, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_offsets, dim3(blocks_for(count)), dim3(kBlock), 0, s, sr * Ly, Lx, dt, step0,
                     count, out);
  return hipGetLastError();
}

hipError_t launch_philox(const uint32_t* ctr, const uint32_t* key, uint32_t* out, int64_t count,
                         hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_philox, dim3(blocks_for(count)), dim3(kBlock), 0, s, ctr, key, out, count);
  return hipGetLastError();
}

}  // namespace le
