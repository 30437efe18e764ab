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

#include "le_internal.h"

namespace le {

// ---------------------------------------------------------------- helpers
__device__ __forceinline__ int xcd_block(int nblocks) {
  // Blocks are dealt round-robin to the 8 XCDs; remap so that each XCD works
  // on one contiguous range of cell-sorted particles (its L2 then holds that
  // region's neighbour positions).
  const int X = 8;
  int b = blockIdx.x;
  int q = nblocks / X, r = nblocks % X;
  int x = b % X, k = b / X;
  return x * q + (x < r ? x : r) + k;
}

__device__ __forceinline__ void latch(Ctrl* c, int32_t st) { atomicCAS(&c->status, 0, st); }

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
    uint32_t lo0 = 0xD2511F53u * c[0];
    uint32_t hi0 = __umulhi(0xD2511F53u, c[0]);
    uint32_t lo1 = 0xCD9E8D57u * c[2];
    uint32_t hi1 = __umulhi(0xCD9E8D57u, c[2]);
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
      d.vel[0][a * np + i] = u0[a * n + i];
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
    c->vmax_bits = 0ull;
    c->pos_cur = 0;
    c->aux_cur = 0;
    c->rebuild = 1;
    c->status = 0;
    c->wraps = 0;
    c->max_nb = 0;
    c->ticket = 0u;
  }
}

// ------------------------------------------------------------- rebuild
// Rebuild kernels run when the device flag asks for it (or `force`), and are
// otherwise empty launches.  Order: wrap+bin, scan (2 kernels), scatter,
// rank+permute, neighbour lists, finish.
__device__ __forceinline__ bool rebuild_off(const Dev& d, int force) {
  const Ctrl* c = d.ctrl;
  return c->status != 0 || !(force || c->rebuild);
}

// Boundary crossing (Lees-Edwards shift and velocity jump) + periodic wrap of
// x and z, then the cell of every particle and its arrival rank in the cell.
__global__ void k_wrap_bin(Dev d, int force) {
  if (rebuild_off(d, force)) return;
  Ctrl* c = d.ctrl;
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) c->max_nb = 0;
  if (i >= d.n) return;
  const int np = d.np;
  double4* P = reinterpret_cast<double4*>(d.pos[c->pos_cur]);
  double* U = d.vel[c->aux_cur];
  double4 p = P[i];
  double x = p.x, y = p.y, z = p.z;
  double ux = U[i];
  const double Delta = c->Delta;
  double ky = wrap1(y, d.Ly);
  x = x - ky * Delta;
  ux = ux - ky * d.sv;
  wrap1(x, d.Lx);
  wrap1(z, d.Lz);
  double uy = U[np + i], uz = U[2 * np + i];
  if (!(isfinite(x) && isfinite(y) && isfinite(z) && isfinite(ux) && isfinite(uy) && isfinite(uz))) {
    latch(c, LE_E_NONFINITE);
    x = 0.0; y = 0.0; z = 0.0;
  }
  p.x = x; p.y = y; p.z = z;
  P[i] = p;
  U[i] = ux;
  int ix = cell_index(x, d.inv_lx, d.nx);
  int iy = cell_index(y, d.inv_ly, d.ny);
  int iz = cell_index(z, d.inv_lz, d.nz);
  int cell = (iz * d.ny + iy) * d.nx + ix;
  d.cell_of[i] = cell;
  d.rank[i] = atomicAdd(&d.cell_count[cell], 1);
}

// Exclusive scan of the cell counts, pass 1: per-chunk scan + chunk totals.
__global__ void k_scan_local(Dev d, int force) {
  if (rebuild_off(d, force)) return;
  __shared__ int wsum[kBlock / 64];
  const int per = kScanChunk / kBlock;  // cells per thread
  int base = blockIdx.x * kScanChunk + threadIdx.x * per;
  int v[per];
  int s = 0;
#pragma unroll
  for (int q = 0; q < per; ++q) {
    int c = base + q;
    v[q] = (c < d.ncell) ? d.cell_count[c] : 0;
    s += v[q];
  }
  // inclusive scan of thread sums across the block
  int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  int incl = s;
  for (int o = 1; o < 64; o <<= 1) {
    int t = __shfl_up(incl, o, 64);
    if (lane >= o) incl += t;
  }
  if (lane == 63) wsum[wid] = incl;
  __syncthreads();
  int woff = 0;
  for (int w = 0; w < wid; ++w) woff += wsum[w];
  int excl = woff + incl - s;
#pragma unroll
  for (int q = 0; q < per; ++q) {
    int c = base + q;
    if (c < d.ncell) d.cell_start[c] = excl;
    excl += v[q];
  }
  if (threadIdx.x == kBlock - 1) d.block_sums[blockIdx.x] = woff + incl;
}

// Pass 2: add the total of all earlier chunks to each chunk.
__global__ void k_scan_add(Dev d, int force, int nchunks) {
  if (rebuild_off(d, force)) return;
  __shared__ int red[kBlock];
  int t = 0;
  for (int b = threadIdx.x; b < (int)blockIdx.x; b += kBlock) t += d.block_sums[b];
  red[threadIdx.x] = t;
  __syncthreads();
  for (int o = kBlock / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  int off = red[0];
  int base = blockIdx.x * kScanChunk;
  for (int q = threadIdx.x; q < kScanChunk; q += kBlock) {
    int c = base + q;
    if (c < d.ncell) d.cell_start[c] += off;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) d.cell_start[d.ncell] = d.n;
  (void)nchunks;
}

__global__ void k_scatter(Dev d, int force) {
  if (rebuild_off(d, force)) return;
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= d.n) return;
  d.src[d.cell_start[d.cell_of[i]] + d.rank[i]] = i;
}

// Deterministic in-cell order: the final slot of a particle is the cell start
// plus the number of cell-mates with a smaller tag.  Gathers every field
// into the other buffer set.
__global__ void k_rank_permute(Dev d, int force) {
  if (rebuild_off(d, force)) return;
  const Ctrl* c = d.ctrl;
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= d.n) return;
  const int np = d.np;
  const int pc = c->pos_cur, ac = c->aux_cur;
  const int32_t* tag = d.tag[ac];
  int i = d.src[p];
  int cell = d.cell_of[i];
  int s0 = d.cell_start[cell], s1 = d.cell_start[cell + 1];
  int t = tag[i];
  int r = 0;
  for (int q = s0; q < s1; ++q) r += (tag[d.src[q]] < t) ? 1 : 0;
  int ns = s0 + r;
  reinterpret_cast<double4*>(d.pos[1 - pc])[ns] = reinterpret_cast<const double4*>(d.pos[pc])[i];
  for (int a = 0; a < 3; ++a) {
    d.vel[1 - ac][a * np + ns] = d.vel[ac][a * np + i];
    d.frc[1 - ac][a * np + ns] = d.frc[ac][a * np + i];
  }
  d.tag[1 - ac][ns] = t;
  d.slot_of_tag[t] = ns;
  d.cell_count[cell] = 0;  // ready for the next binning pass
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
// Cells of one row that are adjacent in memory and share an image are
// scanned as one contiguous slot range, four candidates per batch so that
// several gathers are in flight.  Lists are padded with the sentinel slot n:
// plain entries to a multiple of kPlainBatch, imaged ones to kImgBatch.
constexpr int kPlainBatch = 8;
constexpr int kImgBatch = 4;

__global__ void __launch_bounds__(kBlock) k_neighbors(Dev d, int force) {
  if (rebuild_off(d, force)) return;
  Ctrl* c = d.ctrl;
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= d.n) return;
  const int np = d.np, K = d.K, n = d.n;
  const int pn = 1 - c->pos_cur, an = 1 - c->aux_cur;
  const double4* P = reinterpret_cast<const double4*>(d.pos[pn]);
  const double Delta = c->Delta;
  const double4 pi = P[i];
  const int ix = cell_index(pi.x, d.inv_lx, d.nx);
  const int iy = cell_index(pi.y, d.inv_ly, d.ny);
  const int iz = cell_index(pi.z, d.inv_lz, d.nz);
  const double rl2 = d.rlist2;
  const double rmarg = d.rlist * (1.0 + 1e-12) + 1e-12 * (d.Lx + d.Ly + d.Lz);
  int npl = 0, nim = 0;
  for (int dzc = -1; dzc <= 1; ++dzc) {
    int jz = iz + dzc;
    int sz = jz < 0 ? -1 : (jz >= d.nz ? 1 : 0);
    jz -= sz * d.nz;
    for (int dyc = -1; dyc <= 1; ++dyc) {
      int jy = iy + dyc;
      int sy = jy < 0 ? -1 : (jy >= d.ny ? 1 : 0);
      jy -= sy * d.ny;
      int klo, khi;
      if (sy == 0) {
        klo = ix - 1; khi = ix + 1;
      } else {
        double sh = (double)sy * Delta;
        klo = (int)floor(((double)ix * d.lx - rmarg - sh) / d.lx);
        khi = (int)floor(((double)(ix + 1) * d.lx + rmarg - sh) / d.lx);
      }
      const int rowbase = (jz * d.ny + jy) * d.nx;
      const double shy = (double)sy * d.Ly;
      const double shd = (double)sy * Delta;
      const double shz = (double)sz * d.Lz;
      int k = klo;
      while (k <= khi) {
        // one segment: cells k .. kend with the same x image
        int sx = floor_div(k, d.nx);
        int kend = (sx + 1) * d.nx - 1;
        if (kend > khi) kend = khi;
        const int c0 = rowbase + (k - sx * d.nx);
        const int c1 = rowbase + (kend - sx * d.nx);
        const int q0 = d.cell_start[c0], q1 = d.cell_start[c1 + 1];
        const bool plain = (sx == 0 && sy == 0 && sz == 0);
        const double shx = (double)sx * d.Lx;
        const uint8_t code = pack_img(sx, sy, sz);
        for (int q = q0; q < q1; q += 4) {
          int qq[4];
          double4 pj[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            qq[u] = (q + u < q1) ? q + u : n;
            pj[u] = P[qq[u]];
          }
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            double dy = (pi.y - pj[u].y) - shy;
            double dx = ((pi.x - pj[u].x) - shd) - shx;
            double dz = (pi.z - pj[u].z) - shz;
            double r2 = dx * dx + dy * dy;
            r2 = r2 + dz * dz;
            if (r2 < rl2 && !(plain && qq[u] == i)) {
              if (npl + nim < K) {
                if (plain) {
                  d.nl[npl * np + i] = qq[u];
                } else {
                  int row = K - 1 - nim;
                  d.nl[row * np + i] = qq[u];
                  d.nlc[row * np + i] = code;
                }
              }
              if (plain) ++npl; else ++nim;
            }
          }
        }
        k = kend + 1;
      }
    }
  }
  atomicMax(&c->max_nb, npl + nim);
  // pad both parts to whole batches with the sentinel
  int npl_p = (npl + kPlainBatch - 1) / kPlainBatch * kPlainBatch;
  int nim_p = (nim + kImgBatch - 1) / kImgBatch * kImgBatch;
  if (npl_p + nim_p > K) {
    latch(c, LE_E_CAPACITY);
    npl_p = 0;
    nim_p = 0;
  } else {
    for (int r = npl; r < npl_p; ++r) d.nl[r * np + i] = n;
    const uint8_t zero = pack_img(0, 0, 0);
    for (int r = nim; r < nim_p; ++r) {
      d.nl[(K - 1 - r) * np + i] = n;
      d.nlc[(K - 1 - r) * np + i] = zero;
    }
  }
  d.n_plain[i] = npl_p;
  d.n_img[i] = nim_p;
  if (d.chain_len > 0) {
    int t = d.tag[an][i];
    int lo = -1, hi = -1;
    if (t < d.n_bonded) {
      int kk = t % d.chain_len;
      if (kk > 0) lo = d.slot_of_tag[t - 1];
      if (kk < d.chain_len - 1) hi = d.slot_of_tag[t + 1];
    }
    d.bond[i] = lo;
    d.bond[np + i] = hi;
  }
}

__global__ void k_rebuild_finish(Dev d, int force) {
  if (rebuild_off(d, force)) return;
  Ctrl* c = d.ctrl;
  c->pos_cur ^= 1;
  c->aux_cur ^= 1;
  c->rebuild = 0;
  c->rebuild_step = c->step;
  c->Delta_ref = c->Delta;
  c->drift = 0.0;
  c->wraps = 0;
  c->n_rebuilds += 1;
}

// ---------------------------------------------------------- integrator
__device__ __forceinline__ void vmax_commit(Ctrl* c, double v2) {
  double m = wave_max(v2);
  if ((threadIdx.x & 63) == 0) atomicMax(&c->vmax_bits, (unsigned long long)__double_as_longlong(m));
}

// Advance the step counter and the offset, adopt the new positions, and
// decide whether the neighbour lists must be rebuilt before the next force
// evaluation.  Pair displacements evolve as d' = d + dt (c_i - c_j) +
// gamma_dot dt d_y e_x, so after a strain s = |gamma_dot| (t - t_build) and a
// peculiar path bound D = sum dt max|c|, a pair within rc now was within
// g (rc + 2 g D) at the build, g = s/2 + sqrt(1 + s^2/4) the norm of the
// inverse shear.  The lists (radius rc + skin) stay complete while that bound
// is below rc + skin.  Runs on one thread after every block of the drift
// kernel has finished.
__device__ void control_update(const Dev& d, Ctrl* c) {
  double vmax = sqrt(__longlong_as_double((long long)c->vmax_bits));
  c->vmax_bits = 0ull;
  c->drift += d.dt * vmax;
  c->step += 1;
  c->Delta = le_offset(c->step, d.dt, d.sv, d.Lx);
  c->pos_cur ^= 1;
  double T = (double)(c->step - c->rebuild_step) * d.dt;
  c->wraps = (int)rint((c->Delta_ref + d.sv * T - c->Delta) / d.Lx);
  double s = fabs(d.shear_rate) * T;
  double g = 0.5 * s + sqrt(1.0 + 0.25 * s * s);
  double rc = sqrt(d.rc2);
  double need = g * (rc + 2.0 * g * c->drift);
  if (d.rlist <= rc || need >= d.rlist * (1.0 - 1e-9)) c->rebuild = 1;
}

// Last-block pattern: every block publishes its writes and takes a ticket;
// the block that takes the final ticket sees all of them.  Returns true in
// every thread of that block.
__device__ __forceinline__ bool last_block(Ctrl* c) {
  __shared__ int is_last;
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence();
    unsigned t = atomicAdd(&c->ticket, 1u);
    is_last = (t == gridDim.x - 1) ? 1 : 0;
  }
  __syncthreads();
  if (is_last) __threadfence();
  return is_last != 0;
}

// Sum the per-block stress partials (fixed order) and write the stress
// -(K + W)/V, or with virial_only the pair virial W, into out6.  Called by one
// whole block.
__device__ void reduce_partials(const Dev& d, double* out6, bool virial_only) {
  __shared__ double red[kBlock / 64][kStressComps];
  double acc[kStressComps];
#pragma unroll
  for (int k = 0; k < kStressComps; ++k) acc[k] = 0.0;
  for (int b = threadIdx.x; b < d.nblocks; b += kBlock) {
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
// u += dt/(2m) F ; x_new = x + dt u (into the other position buffer); the
// last block then advances the step (control_update).
__global__ void __launch_bounds__(kBlock) k_kick_drift(Dev d) {
  __shared__ int skip;
  Ctrl* c = d.ctrl;
  if (threadIdx.x == 0) skip = c->status;
  __syncthreads();
  if (skip) return;
  int i = blockIdx.x * blockDim.x + threadIdx.x;
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
    double cx = ux - d.shear_rate * (p.y - 0.5 * d.Ly);
    v2 = cx * cx + uy * uy + uz * uz;
    U[i] = ux; U[np + i] = uy; U[2 * np + i] = uz;
    double4 q;
    q.x = p.x + d.dt * ux;
    q.y = p.y + d.dt * uy;
    q.z = p.z + d.dt * uz;
    q.w = p.w;
    reinterpret_cast<double4*>(d.pos[1 - pc])[i] = q;
    if (!(isfinite(q.x) && isfinite(q.y) && isfinite(q.z))) latch(c, LE_E_NONFINITE);
  }
  vmax_commit(c, v2);
  if (last_block(c) && threadIdx.x == 0) {
    control_update(d, c);
    c->ticket = 0u;
  }
}

// ---------------------------------------------------------- force kernel
template <bool VIR>
__device__ __forceinline__ void add_pair(double f, double dx, double dy, double dz, double& fx,
                                         double& fy, double& fz, double* w) {
  double ax = f * dx, ay = f * dy, az = f * dz;
  fx += ax; fy += ay; fz += az;
  if (VIR) {
    w[0] = fma(dx, ax, w[0]); w[1] = fma(dy, ay, w[1]); w[2] = fma(dz, az, w[2]);
    w[3] = fma(dx, ay, w[3]); w[4] = fma(dx, az, w[4]); w[5] = fma(dy, az, w[5]);
  }
}

template <bool MIXED>
__device__ __forceinline__ double lj_scalar(double r2, double sig2, double eps24) {
  if (MIXED) {
    float r2f = (float)r2;
    float inv = __builtin_amdgcn_rcpf(r2f);
    inv = inv * (2.0f - r2f * inv);  // one Newton step: ~1 ulp
    float s2 = (float)sig2 * inv;
    float s6 = s2 * s2 * s2;
    return (double)((float)eps24 * s6 * (2.0f * s6 - 1.0f) * inv);
  } else {
    double inv = 1.0 / r2;
    double s2 = sig2 * inv;
    double s6 = s2 * s2 * s2;
    return eps24 * s6 * fma(2.0, s6, -1.0) * inv;
  }
}

// Block reduction of 12 per-thread sums into partials[block][12] (fixed
// order: wave butterflies, then waves in index order).
__device__ __forceinline__ void block_partials(double* vals, double* out, int lb) {
  __shared__ double red[kBlock / 64][kStressComps];
  int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < kStressComps; ++k) {
    double v = vals[k];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if (lane == 0) red[wid][k] = v;
  }
  __syncthreads();
  if (threadIdx.x < kStressComps) {
    double s = 0.0;
    for (int w = 0; w < kBlock / 64; ++w) s += red[w][threadIdx.x];
    out[lb * kStressComps + threadIdx.x] = s;
  }
}

// One evaluation of the conservative force for every particle, and then,
// depending on MODE:
//   kForcesOnly  write F^c in tag order (+ kinetic and virial partials)
//   kInitForce   F = F^c + Langevin(u) of the current step into frc
//   kStepLast    F as above from the half-step velocity, u += dt/(2m) F
//   kStepFused   as kStepLast, then the next half-kick and drift
// Langevin force (Eq. langevin on the peculiar velocity, Eq. vi):
//   F = F^c - gamma m c + sqrt(24 gamma m kT / dt) theta,  c = u - gamma_dot (y - L_y/2) e_x
template <int MODE, bool MIXED, bool BONDS, bool SAMPLE>
__global__ void __launch_bounds__(kBlock) k_force(Dev d, double* __restrict__ f_out,
                                                  double* __restrict__ sample_out) {
  constexpr bool VIR = SAMPLE || (MODE == kForcesOnly);
  __shared__ int skip;
  Ctrl* c = d.ctrl;
  if (threadIdx.x == 0) skip = c->status;
  __syncthreads();
  if (skip) return;
  const int lb = xcd_block(d.nblocks);
  const int i = lb * kBlock + threadIdx.x;
  const bool valid = i < d.n;
  const int np = d.np, K = d.K;
  const int pc = c->pos_cur, ac = c->aux_cur;
  const double Delta = c->Delta;
  const int W = c->wraps;
  const double4* P = reinterpret_cast<const double4*>(d.pos[pc]);
  double fx = 0.0, fy = 0.0, fz = 0.0;
  double w[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  double4 pi = make_double4(0.0, 0.0, 0.0, 0.0);
  if (valid) {
    pi = P[i];
    const double rc2 = d.rc2, sig2 = d.sig2, eps24 = d.eps24;
    const int npl = d.n_plain[i];  // a multiple of kPlainBatch (sentinel-padded)
    const int* __restrict__ nl = d.nl + i;
    int jn[kPlainBatch];
    if (npl > 0) {
#pragma unroll
      for (int u = 0; u < kPlainBatch; ++u) jn[u] = nl[u * np];
    }
    for (int k = 0; k < npl; k += kPlainBatch) {
      double4 pj[kPlainBatch];
#pragma unroll
      for (int u = 0; u < kPlainBatch; ++u) pj[u] = P[jn[u]];
      if (k + kPlainBatch < npl) {
#pragma unroll
        for (int u = 0; u < kPlainBatch; ++u) jn[u] = nl[(k + kPlainBatch + u) * np];
      }
#pragma unroll
      for (int u = 0; u < kPlainBatch; ++u) {
        double dx = pi.x - pj[u].x, dy = pi.y - pj[u].y, dz = pi.z - pj[u].z;
        double r2 = dx * dx + dy * dy;
        r2 = r2 + dz * dz;
        if (r2 < rc2) add_pair<VIR>(lj_scalar<MIXED>(r2, sig2, eps24), dx, dy, dz, fx, fy, fz, w);
      }
    }
    const int nim = d.n_img[i];  // a multiple of kImgBatch
    for (int k = 0; k < nim; k += kImgBatch) {
      int jj[kImgBatch];
      uint8_t cc[kImgBatch];
      double4 pj[kImgBatch];
#pragma unroll
      for (int u = 0; u < kImgBatch; ++u) {
        int row = K - 1 - (k + u);
        jj[u] = nl[row * np];
        cc[u] = d.nlc[row * np + i];
      }
#pragma unroll
      for (int u = 0; u < kImgBatch; ++u) pj[u] = P[jj[u]];
#pragma unroll
      for (int u = 0; u < kImgBatch; ++u) {
        int sx, sy, sz;
        unpack_img(cc[u], sx, sy, sz);
        sx += sy * W;
        double dy = (pi.y - pj[u].y) - (double)sy * d.Ly;
        double dx = ((pi.x - pj[u].x) - (double)sy * Delta) - (double)sx * d.Lx;
        double dz = (pi.z - pj[u].z) - (double)sz * d.Lz;
        double r2 = dx * dx + dy * dy;
        r2 = r2 + dz * dz;
        if (r2 < rc2) add_pair<VIR>(lj_scalar<MIXED>(r2, sig2, eps24), dx, dy, dz, fx, fy, fz, w);
      }
    }
    if (BONDS) {
      // FENE (Eq. fene), always float64; displacement by the nearest image
      for (int b = 0; b < 2; ++b) {
        int j = d.bond[b * np + i];
        if (j < 0) continue;
        double4 pj = P[j];
        double dy0 = pi.y - pj.y;
        double sy = rint(dy0 / d.Ly);
        double dy = dy0 - sy * d.Ly;
        double dx0 = (pi.x - pj.x) - sy * Delta;
        double sx = rint(dx0 / d.Lx);
        double dx = dx0 - sx * d.Lx;
        double dz0 = pi.z - pj.z;
        double sz = rint(dz0 / d.Lz);
        double dz = dz0 - sz * d.Lz;
        double r2 = dx * dx + dy * dy;
        r2 = r2 + dz * dz;
        if (!(r2 < d.fene_r02)) {
          latch(c, LE_E_BOND);
          continue;
        }
        double f = -d.fene_k / (1.0 - r2 / d.fene_r02);
        add_pair<VIR>(f, dx, dy, dz, fx, fy, fz, w);
      }
    }
  }
  double kin[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  double v2 = 0.0;
  if (MODE == kForcesOnly) {
    if (valid) {
      int t = d.tag[ac][i];
      if (f_out) {
        f_out[t] = fx; f_out[d.n + t] = fy; f_out[2 * d.n + t] = fz;
      }
      const double* U = d.vel[ac];
      double cx = U[i] - d.shear_rate * (pi.y - 0.5 * d.Ly);
      double cy = U[np + i], cz = U[2 * np + i];
      double m = d.mass;
      kin[0] = m * cx * cx; kin[1] = m * cy * cy; kin[2] = m * cz * cz;
      kin[3] = m * cx * cy; kin[4] = m * cx * cz; kin[5] = m * cy * cz;
    }
  } else if (valid) {
    double* U = d.vel[ac];
    double ux = U[i], uy = U[np + i], uz = U[2 * np + i];
    int t = d.tag[ac][i];
    uint32_t ctr[4] = {(uint32_t)(uint64_t)c->step, (uint32_t)((uint64_t)c->step >> 32), (uint32_t)t, 0u};
    philox(ctr, d.seed_lo, d.seed_hi);
    double cx = ux - d.shear_rate * (pi.y - 0.5 * d.Ly);
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
        double cxn = ux - d.shear_rate * (pi.y - 0.5 * d.Ly);
        kin[0] = m * cxn * cxn; kin[1] = m * uy * uy; kin[2] = m * uz * uz;
        kin[3] = m * cxn * uy; kin[4] = m * cxn * uz; kin[5] = m * uy * uz;
      }
      if (MODE == kStepLast) {
        double* F = d.frc[ac];
        F[i] = Fx; F[np + i] = Fy; F[2 * np + i] = Fz;
      } else {
        ux = ux + d.h * Fx; uy = uy + d.h * Fy; uz = uz + d.h * Fz;
        double cxh = ux - d.shear_rate * (pi.y - 0.5 * d.Ly);
        v2 = cxh * cxh + uy * uy + uz * uz;
        double4 q;
        q.x = pi.x + d.dt * ux;
        q.y = pi.y + d.dt * uy;
        q.z = pi.z + d.dt * uz;
        q.w = pi.w;
        reinterpret_cast<double4*>(d.pos[1 - pc])[i] = q;
        if (!(isfinite(q.x) && isfinite(q.y) && isfinite(q.z))) latch(c, LE_E_NONFINITE);
      }
      U[i] = ux; U[np + i] = uy; U[2 * np + i] = uz;
    }
  }
  if (MODE == kStepFused) vmax_commit(c, v2);
  if (VIR) {
    double vals[kStressComps];
#pragma unroll
    for (int k = 0; k < 6; ++k) { vals[k] = kin[k]; vals[6 + k] = 0.5 * w[k]; }
    block_partials(vals, d.partials, lb);
  }
  if (MODE == kStepFused || (MODE == kStepLast && SAMPLE)) {
    if (last_block(c)) {
      if (SAMPLE) reduce_partials(d, sample_out, false);
      if (threadIdx.x == 0) {
        if (MODE == kStepFused) control_update(d, c);
        c->ticket = 0u;
      }
    }
  }
}

// Stand-alone reduction of the block partials (le_forces, le_stress).
__global__ void k_stress_final(Dev d, double* out6, int virial_only) {
  __shared__ int skip;
  if (threadIdx.x == 0) skip = d.ctrl->status;
  __syncthreads();
  if (skip) return;
  reduce_partials(d, out6, virial_only != 0);
}

// ----------------------------------------------------------- state out
__global__ void k_state_out(Dev d, double* x, double* u, int32_t* cell_of, int32_t* order) {
  if (d.ctrl->status) return;
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
  if (d.ctrl->status) return;
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= d.n) return;
  const int np = d.np, K = d.K;
  const int32_t* tag = d.tag[d.ctrl->aux_cur];
  int ti = tag[i];
  int npl = d.n_plain[i], nim = d.n_img[i];
  for (int k = 0; k < npl + nim; ++k) {
    int row = k < npl ? k : K - 1 - (k - npl);
    int tj = tag[d.nl[row * np + i]];
    if (ti < tj) {
      unsigned long long idx = atomicAdd(counter, 1ull);
      if ((int64_t)idx < cap) { pairs[2 * idx] = ti; pairs[2 * idx + 1] = tj; }
    }
  }
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

hipError_t launch_rebuild(const Dev& d, hipStream_t s, bool force) {
  int f = force ? 1 : 0;
  int nb = blocks_for(d.n);
  int nchunks = (d.ncell + kScanChunk - 1) / kScanChunk;
  hipLaunchKernelGGL(k_wrap_bin, dim3(nb), dim3(kBlock), 0, s, d, f);
  hipLaunchKernelGGL(k_scan_local, dim3(nchunks), dim3(kBlock), 0, s, d, f);
  hipLaunchKernelGGL(k_scan_add, dim3(nchunks), dim3(kBlock), 0, s, d, f, nchunks);
  hipLaunchKernelGGL(k_scatter, dim3(nb), dim3(kBlock), 0, s, d, f);
  hipLaunchKernelGGL(k_rank_permute, dim3(nb), dim3(kBlock), 0, s, d, f);
  hipLaunchKernelGGL(k_neighbors, dim3(nb), dim3(kBlock), 0, s, d, f);
  hipLaunchKernelGGL(k_rebuild_finish, dim3(1), dim3(1), 0, s, d, f);
  return hipGetLastError();
}

hipError_t launch_kick_drift(const Dev& d, hipStream_t s) {
  hipLaunchKernelGGL(k_kick_drift, dim3(blocks_for(d.n)), dim3(kBlock), 0, s, d);
  return hipGetLastError();
}

template <int MODE, bool SAMPLE>
static void launch_force_t(const Dev& d, hipStream_t s, double* f_out, double* so) {
  dim3 g(d.nblocks), b(kBlock);
  const bool bonds = d.chain_len > 0;
  const bool mixed = d.precision == LE_MIXED;
  if (mixed) {
    if (bonds) hipLaunchKernelGGL((k_force<MODE, true, true, SAMPLE>), g, b, 0, s, d, f_out, so);
    else hipLaunchKernelGGL((k_force<MODE, true, false, SAMPLE>), g, b, 0, s, d, f_out, so);
  } else {
    if (bonds) hipLaunchKernelGGL((k_force<MODE, false, true, SAMPLE>), g, b, 0, s, d, f_out, so);
    else hipLaunchKernelGGL((k_force<MODE, false, false, SAMPLE>), g, b, 0, s, d, f_out, so);
  }
}

hipError_t launch_force(const Dev& d, hipStream_t s, ForceMode mode, bool sample, double* f_out,
                        double* sample_out) {
  switch (mode) {
    case kForcesOnly: launch_force_t<kForcesOnly, false>(d, s, f_out, nullptr); break;
    case kInitForce: launch_force_t<kInitForce, false>(d, s, f_out, nullptr); break;
    case kStepLast:
      if (sample) launch_force_t<kStepLast, true>(d, s, f_out, sample_out);
      else launch_force_t<kStepLast, false>(d, s, f_out, nullptr);
      break;
    case kStepFused:
      if (sample) launch_force_t<kStepFused, true>(d, s, f_out, sample_out);
      else launch_force_t<kStepFused, false>(d, s, f_out, nullptr);
      break;
  }
  return hipGetLastError();
}

hipError_t launch_stress_final(const Dev& d, hipStream_t s, double* out6, bool virial_only) {
  hipLaunchKernelGGL(k_stress_final, dim3(1), dim3(kBlock), 0, s, d, out6, virial_only ? 1 : 0);
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
