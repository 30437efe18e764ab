// le_api.hip -- host side of the C ABI declared in include/le.h: parameter
// validation, workspace carving, and the launch sequence of each entry point.
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <mutex>
#include <new>
#include <vector>

#include "le_internal.h"

using namespace le;

struct le_graph {
  hipStream_t stream;
  hipGraph_t graph;
  hipGraphExec_t exec;
  std::vector<le_sim*> sims;  // the simulations it advances (one, or a batch)
  std::vector<Ctrl*> ctrl_at; // each one's control copy current when the graph starts
};

struct le_sim {
  le_params p;
  Dev d;
  hipStream_t stream;
  int32_t host_status;                 // last status seen by a synchronising call
  Ctrl* ctrl_base;                     // the two control copies; d.ctrl is the current one
  unsigned long long* vmax_base;       // the two speed-bound slot arrays (d.vmax current)
  Dev* dev_dev;                         // device copies of d for the two control copies (batched launches)
  unsigned long long* counter;         // device scratch counter (pairs_out)
  double* scratch6;                    // device 6 doubles
  // phase timing (le_timing_enable)
  int32_t timing;                      // bit k: time phase k
  int32_t timing_stride;               // time every timing_stride-th plain-step force launch
  uint64_t tick;                       // plain-step force launches since enabling
  std::vector<hipEvent_t> ev;          // pairs (start, stop)
  std::vector<int> ev_phase;           // phase of each recorded pair
  size_t ev_used;                      // pairs recorded and not yet folded
  double phase_ms[4];
  int64_t phase_n[4];
};

namespace {

constexpr size_t kAlign = 256;

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

struct Geometry {
  int32_t nc[3];
  double rc, rlist;
  int32_t K;
  int64_t np;
  int32_t nblocks;
  int32_t bcap;
  int32_t sp_cells, sp_blocks;  // scan-and-permute pass: cells per block, blocks
};

le_status validate(const le_params* p, Geometry* g) {
  if (!p) return LE_E_ARG;
  // slots (n + 1 with the sentinel) share a 32-bit list entry with a 7-bit image code
  if (p->n < 2 || p->n >= ((int64_t)1 << kSlotBits) - 1) return LE_E_ARG;
  for (int a = 0; a < 3; ++a)
    if (!(p->box[a] > 0.0) || !isfinite(p->box[a])) return LE_E_ARG;
  if (!(p->dt > 0.0) || !(p->mass > 0.0) || !(p->kT >= 0.0) || !(p->gamma >= 0.0)) return LE_E_ARG;
  if (!isfinite(p->shear_rate) || !(p->sigma > 0.0) || !(p->skin >= 0.0) || !isfinite(p->eps))
    return LE_E_ARG;
  if (p->pair != LE_PAIR_LJ && p->pair != LE_PAIR_WCA) return LE_E_ARG;
  if (p->precision != LE_FP64 && p->precision != LE_MIXED) return LE_E_ARG;
  if (p->tune < 0 || p->tune > 2) return LE_E_ARG;
  if (p->thermostat < LE_THERMO_LANGEVIN || p->thermostat > LE_THERMO_LANGEVIN_LAB) return LE_E_ARG;
  if (p->velocity != LE_VEL_LAB && p->velocity != LE_VEL_PECULIAR) return LE_E_ARG;
  // peculiar storage is defined with the Langevin force on the stored velocity
  if (p->velocity == LE_VEL_PECULIAR && p->thermostat != LE_THERMO_LANGEVIN) return LE_E_ARG;
  double rc = p->rc;
  if (rc <= 0.0) rc = (p->pair == LE_PAIR_WCA) ? pow(2.0, 1.0 / 6.0) * p->sigma : 2.5 * p->sigma;
  if (p->thermostat == LE_THERMO_DPD) {
    // the pair terms run over the neighbour lists (radius rc + skin, valid
    // for r < rc), in the global-memory layout
    if (!(p->dpd_rc >= 0.0) || p->dpd_rc > rc || p->tune == 1) return LE_E_ARG;
  }
  if (!(p->force_cap >= 0.0) || !isfinite(p->force_cap)) return LE_E_ARG;
  if (p->force_cap > 0.0 && (p->precision != LE_FP64 || p->thermostat == LE_THERMO_DPD || p->tune == 1))
    return LE_E_ARG;  // the capped force law exists for the FP64 global-memory layout
  if (p->chain_len < 0 || p->n_chains < 0) return LE_E_ARG;
  if (p->n_chains > 0) {
    if (p->chain_len < 2 || p->n_chains * (int64_t)p->chain_len > p->n) return LE_E_ARG;
    if (!(p->fene_r0 > 0.0) || !(p->fene_k >= 0.0)) return LE_E_ARG;
    if (!(p->angle_k >= 0.0) || !isfinite(p->angle_k)) return LE_E_ARG;
  }
  double rlist = rc + p->skin;
  for (int a = 0; a < 3; ++a) {
    int32_t k = p->cells[a];
    if (k <= 0) k = (int32_t)floor(p->box[a] / (rlist * (1.0 + 1e-9)));
    if (k < 3) return LE_E_GEOMETRY;
    if (p->box[a] / k < rlist) return LE_E_GEOMETRY;
    if ((int64_t)k * k * k > (int64_t)1 << 30) return LE_E_GEOMETRY;
    g->nc[a] = k;
  }
  if ((int64_t)g->nc[0] * g->nc[1] * g->nc[2] > (int64_t)0x7fffffff - 1) return LE_E_GEOMETRY;
  g->rc = rc;
  g->rlist = rlist;
  // capacity of each of a particle's two sub-lists (each holds about half of
  // its partners; the first also the second's partial last block):
  // max_neighbors / 2, or from the density with a margin
  if (p->max_neighbors > 0) {
    g->K = (p->max_neighbors + 1) / 2;
  } else {
    double rho = (double)p->n / (p->box[0] * p->box[1] * p->box[2]);
    double mean = 4.0 / 3.0 * M_PI * rlist * rlist * rlist * rho;
    g->K = (int32_t)ceil(mean) + 40;
  }
  if (g->K > 4096) g->K = 4096;
  g->K = (g->K + 7) / 8 * 8;  // lists are stored in blocks of 8 (plain) and 4 (other) entries
  g->np = (p->n + 1 + kBlock - 1) / kBlock * kBlock;  // +1: sentinel slot
  {
    // bucket capacity: generous over the mean cell occupancy
    double mean = (double)p->n / ((double)g->nc[0] * g->nc[1] * g->nc[2]);
    double cap = fmin(4.0 * mean + 32.0, (double)p->n);
    g->bcap = ((int32_t)ceil(cap) + 7) / 8 * 8;
  }
  g->nblocks = (int32_t)((p->n + kTile - 1) / kTile);
  {
    // about kSortParticles particles per block of the scan-and-permute pass
    const int64_t ncell = (int64_t)g->nc[0] * g->nc[1] * g->nc[2];
    const double mean = (double)p->n / (double)ncell;
    g->sp_cells = (int32_t)fmin(fmax(ceil(kSortParticles / mean), 1.0), (double)kBlock);
    g->sp_blocks = (int32_t)((ncell + g->sp_cells - 1) / g->sp_cells);
  }
  return LE_OK;
}

// Carve the workspace; with base == nullptr only the size is computed.
size_t carve(const le_params* p, const Geometry& g, char* base, Dev* d, le_sim* s) {
  size_t off = 0;
  auto take = [&](size_t bytes) -> char* {
    char* r = base ? base + off : nullptr;
    off = align_up(off + bytes);
    return r;
  };
  const size_t np = (size_t)g.np;
  const size_t ncell = (size_t)g.nc[0] * g.nc[1] * g.nc[2];
  Dev t;
  memset(&t, 0, sizeof(t));
  t.ctrl = (Ctrl*)take(2 * sizeof(Ctrl));
  t.flags = (Flags*)take(sizeof(Flags));
  t.vmax = (unsigned long long*)take(2 * kSlots * kLineU64 * sizeof(unsigned long long));
  t.scan_status = (unsigned long long*)take((size_t)g.sp_blocks * sizeof(unsigned long long));
  for (int b = 0; b < 2; ++b) {
    t.pos[b] = (double*)take(4 * np * sizeof(double));
    t.vel[b] = (double*)take(3 * np * sizeof(double));
    t.frc[b] = (double*)take(3 * np * sizeof(double));
    t.tag[b] = (int32_t*)take(np * sizeof(int32_t));
  }
  t.vt = (p->thermostat == LE_THERMO_DPD) ? (double*)take(4 * np * sizeof(double)) : nullptr;
  t.slot_of_tag = (int32_t*)take(np * sizeof(int32_t));
  t.bucket = (int2*)take(ncell * (size_t)g.bcap * sizeof(int2));
  t.cell_count = (int32_t*)take(ncell * sizeof(int32_t));
  t.cell_start = (int32_t*)take((ncell + 1) * sizeof(int32_t));
  t.nl16 = (uint16_t*)take((size_t)g.K * 2 * np * sizeof(uint16_t));
  t.nlo = (uint32_t*)take((size_t)g.K * 2 * np * sizeof(uint32_t));
  t.n_plain = (int32_t*)take(2 * np * sizeof(int32_t));
  t.n_og = (int32_t*)take(2 * np * sizeof(int32_t));
  t.halo_slot = (int32_t*)take((size_t)g.nblocks * kHalo * sizeof(int32_t));
  t.halo_code = (uint8_t*)take((size_t)g.nblocks * kHalo);
  t.tile_nstage = (int32_t*)take((size_t)g.nblocks * sizeof(int32_t));
  t.bond = (p->chain_len > 0) ? (int32_t*)take(2 * np * sizeof(int32_t)) : nullptr;
  t.partials = (double*)take((size_t)g.nblocks * kStressComps * sizeof(double));
  t.obs_part = (double*)take((size_t)((p->n + kBlock - 1) / kBlock) * (3 * LE_MAX_BINS + 4) *
                             sizeof(double));
  unsigned long long* counter = (unsigned long long*)take(sizeof(unsigned long long));
  double* scratch6 = (double*)take(6 * sizeof(double));
  Dev* dev_dev = (Dev*)take(2 * sizeof(Dev));
  if (d) {
    // copy buffer pointers into d (geometry fields are filled by the caller)
    d->ctrl = t.ctrl;
    d->flags = t.flags;
    d->vmax = t.vmax;
    d->scan_status = t.scan_status;
    for (int b = 0; b < 2; ++b) {
      d->pos[b] = t.pos[b]; d->vel[b] = t.vel[b]; d->frc[b] = t.frc[b]; d->tag[b] = t.tag[b];
    }
    d->vt = t.vt;
    d->slot_of_tag = t.slot_of_tag; d->bucket = t.bucket;
    d->cell_count = t.cell_count; d->cell_start = t.cell_start;
    d->nl16 = t.nl16; d->nlo = t.nlo;
    d->n_plain = t.n_plain; d->n_og = t.n_og;
    d->halo_slot = t.halo_slot; d->halo_code = t.halo_code; d->tile_nstage = t.tile_nstage;
    d->bond = t.bond;
    d->partials = t.partials;
    d->obs_part = t.obs_part;
  }
  if (s) {
    s->counter = counter;
    s->scratch6 = scratch6;
    s->ctrl_base = t.ctrl;
    s->vmax_base = t.vmax;
    s->dev_dev = dev_dev;
  }
  return off + kAlign;  // room to align the caller's base pointer
}

void fill_geometry(const le_params* p, const Geometry& g, Dev* d) {
  d->Lx = p->box[0]; d->Ly = p->box[1]; d->Lz = p->box[2];
  d->nx = g.nc[0]; d->ny = g.nc[1]; d->nz = g.nc[2];
  d->ncell = g.nc[0] * g.nc[1] * g.nc[2];
  d->inv_lx = (double)g.nc[0] / p->box[0];
  d->inv_ly = (double)g.nc[1] / p->box[1];
  d->inv_lz = (double)g.nc[2] / p->box[2];
  d->lx = p->box[0] / (double)g.nc[0];
  d->shear_rate = p->shear_rate;
  d->sv = p->shear_rate * p->box[1];
  const bool pec = p->velocity == LE_VEL_PECULIAR;
  d->c_sr = pec ? 0.0 : p->shear_rate;
  d->drift_sr = pec ? p->shear_rate : 0.0;
  d->jump_sv = pec ? 0.0 : d->sv;
  d->dt = p->dt;
  d->h = 0.5 * p->dt / p->mass;
  d->gamma_m = p->gamma * p->mass;
  d->pref = sqrt(24.0 * p->gamma * p->mass * p->kT / p->dt);
  d->thermostat = p->thermostat;
  {
    const double dpd_rc = p->dpd_rc > 0.0 ? p->dpd_rc : g.rc;
    d->dpd_gamma = p->gamma;
    d->dpd_pref = sqrt(24.0 * p->gamma * p->kT / p->dt);
    d->dpd_rc2 = dpd_rc * dpd_rc;
    d->dpd_inv_rc = 1.0 / dpd_rc;
  }
  d->mass = p->mass;
  d->eps24 = 24.0 * p->eps;
  d->sig2 = p->sigma * p->sigma;
  d->rc2 = g.rc * g.rc;
  d->rlist = g.rlist;
  d->rlist2 = g.rlist * g.rlist;
  {
    // Bound on |r2_f32 - r2_f64| for a pair near the list radius.  Staged
    // coordinates are relative to a tile particle and image-shifted, so each
    // lies within 4 L_max + r_list of zero; rounding each to float moves it by
    // at most 2^-24 of that, a displacement component by delta = twice that,
    // r2 by 2 sqrt(3) (r_list + delta) delta + 3 delta^2, and the three float
    // operations forming r2 add 3 ulps of r_list^2.  Doubled for safety.
    const double lmax = fmax(p->box[0], fmax(p->box[1], p->box[2]));
    const double u = ldexp(1.0, -24);
    const double delta = 2.0 * u * (4.0 * lmax + g.rlist);
    const double rl2 = g.rlist * g.rlist;
    const double margin = 2.0 * (2.0 * sqrt(3.0) * (g.rlist + delta) * delta + 3.0 * delta * delta +
                                 4.0 * u * rl2 * 1.01) + 1e-12 * rl2;
    d->nb_lo = nextafterf((float)(rl2 - margin), 0.0f);
    d->nb_hi = nextafterf((float)(rl2 + margin), INFINITY);
    if ((double)d->nb_lo + margin > rl2) d->nb_lo = nextafterf(d->nb_lo, 0.0f);
    if ((double)d->nb_hi - margin < rl2) d->nb_hi = nextafterf(d->nb_hi, INFINITY);
  }
  d->fene_k = p->fene_k;
  d->fene_r02 = p->fene_r0 * p->fene_r0;
  d->angle_k = (p->n_chains > 0 && p->chain_len >= 3) ? p->angle_k : 0.0;
  d->force_cap = p->force_cap;
  d->inv_vol = 1.0 / (p->box[0] * p->box[1] * p->box[2]);
  d->n = (int32_t)p->n;
  d->np = (int32_t)g.np;
  d->K = g.K;
  d->np2 = (int32_t)(2 * g.np);
  d->chain_len = p->n_chains > 0 ? p->chain_len : 0;
  d->n_bonded = (int32_t)(p->n_chains * (int64_t)p->chain_len);
  d->precision = p->precision;
  d->seed_lo = (uint32_t)p->seed;
  d->seed_hi = (uint32_t)(p->seed >> 32);
  d->dpd_key_hi = d->seed_hi ^ 0x44504421u;
  d->nblocks = g.nblocks;
  d->ntiles = g.nblocks;
  d->bcap = g.bcap;
  d->sp_cells = g.sp_cells;
  d->sp_blocks = g.sp_blocks;
  {
    // LDS halo at force time when partners per particle clearly outnumber the
    // positions a tile must stage per particle (strip tile of kTile particles:
    // 9 neighbouring rows of (tile cells + 2) cells)
    const double rho = (double)p->n / (p->box[0] * p->box[1] * p->box[2]);
    const double cell_n = rho * (p->box[0] / g.nc[0]) * (p->box[1] / g.nc[1]) * (p->box[2] / g.nc[2]);
    const double tile_cells = kTile / fmax(cell_n, 1e-9);
    const double halo_pp = 9.0 * (tile_cells + 2.0) * cell_n / kTile;
    const double list_pp = 4.0 / 3.0 * M_PI * g.rlist * g.rlist * g.rlist * rho;
    d->staged = (p->tune == 1) ? 1 : (p->tune == 2) ? 0 : (list_pp >= 3.0 * halo_pp ? 1 : 0);
    if (p->thermostat == LE_THERMO_DPD || p->force_cap > 0.0) d->staged = 0;
    // a sparse system's tile halo (with a margin) fits the smaller search
    // halo, which leaves room for more resident blocks
    d->small_halo = (!d->staged && 1.15 * halo_pp * kTile <= kHaloSearch) ? 1 : 0;
  }
}

le_status hip_check(hipError_t e) { return e == hipSuccess ? LE_OK : LE_E_HIP; }

constexpr size_t kMaxEventPairs = 16384;

// Fold recorded event pairs into the per-phase totals (waits for the stream).
le_status fold_events(le_sim* s) {
  if (s->ev_used == 0) return LE_OK;
  if (hipStreamSynchronize(s->stream) != hipSuccess) return LE_E_HIP;
  for (size_t k = 0; k < s->ev_used; ++k) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, s->ev[2 * k], s->ev[2 * k + 1]) != hipSuccess) return LE_E_HIP;
    s->phase_ms[s->ev_phase[k]] += ms;
    s->phase_n[s->ev_phase[k]] += 1;
  }
  s->ev_used = 0;
  return LE_OK;
}

// Reserve an event pair for a timed launch of `phase`; returns its index or
// -1 when the phase is not timed.
long reserve_pair(le_sim* s, int phase) {
  if (!((s->timing >> phase) & 1)) return -1;
  if (s->ev_used == kMaxEventPairs && fold_events(s) != LE_OK) return -1;
  size_t k = s->ev_used;
  if (s->ev.size() < 2 * (k + 1)) {
    hipEvent_t a, b;
    if (hipEventCreate(&a) != hipSuccess) return -1;
    if (hipEventCreate(&b) != hipSuccess) { (void)hipEventDestroy(a); return -1; }
    s->ev.push_back(a);
    s->ev.push_back(b);
    s->ev_phase.push_back(0);
  }
  s->ev_phase[k] = phase;
  return (long)k;
}

// Record the start of a timed launch group; returns the pair index or -1.
long begin_phase(le_sim* s, int phase) {
  long k = reserve_pair(s, phase);
  if (k < 0) return -1;
  if (hipEventRecord(s->ev[2 * k], s->stream) != hipSuccess) return -1;
  return k;
}

void end_phase(le_sim* s, long k) {
  if (k < 0) return;
  if (hipEventRecord(s->ev[2 * k + 1], s->stream) == hipSuccess) s->ev_used = (size_t)k + 1;
}

// Rebuild chain; afterwards the other control copy is the current one.
le_status rebuild(le_sim* s, bool force, bool control) {
  const bool first = s->d.ctrl == s->ctrl_base;
  Ctrl* next = first ? s->ctrl_base + 1 : s->ctrl_base;
  unsigned long long* next_vmax = s->vmax_base + (first ? kSlots * kLineU64 : 0);
  le_status st = hip_check(launch_rebuild(s->d, next, next_vmax, s->stream, force, control));
  s->d.ctrl = next;
  s->d.vmax = next_vmax;
  return st;
}

le_status read_status(le_sim* s) {
  int32_t st = 0;
  if (hipStreamSynchronize(s->stream) != hipSuccess) return LE_E_HIP;
  if (hipMemcpy(&st, &s->d.flags->status, sizeof(st), hipMemcpyDeviceToHost) != hipSuccess)
    return LE_E_HIP;
  if (st != 0) s->host_status = st;
  return s->host_status;
}

// ---------------------------------------------------------------------------
// Library-owned device scratch for le_forces_static: one array per GPU, held
// from module load until the process ends.  In host code `scratch` is only a
// stand-in for the symbol; its device address on the current GPU comes from
// hipGetSymbolAddress, taken once per device and kept in scratch_addr.
constexpr size_t kStaticScratchBytes = (size_t)64 << 20;
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_addr[kMaxDevices] = {};

}  // namespace

static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {

// ---------------------------------------------------------------------------
// Batched stepping: simulations that share a kernel configuration form a
// group; each step launches every kernel once per group (at most kMaxBatch
// simulations per launch), the blocks of all members in one grid.

struct BatchGroup {
  Dev cfg;                     // host descriptor of the first member (kernel configuration)
  std::vector<le_sim*> sims;
  Batch par[2], bin[2], scan[2], tile[2], one[2];  // [v]: v = 0 descriptors of the copies current at the call
};

bool same_config(const Dev& a, const Dev& b) {
  return a.staged == b.staged && a.small_halo == b.small_halo && a.precision == b.precision &&
         (a.chain_len > 0) == (b.chain_len > 0) && (a.force_cap > 0.0) == (b.force_cap > 0.0) &&
         (a.thermostat == LE_THERMO_DPD) == (b.thermostat == LE_THERMO_DPD);
}

void fill_group(BatchGroup& g) {
  for (int v = 0; v < 2; ++v) {
    Batch* bs[5] = {&g.par[v], &g.bin[v], &g.scan[v], &g.tile[v], &g.one[v]};
    for (Batch* b : bs) {
      memset(b, 0, sizeof(Batch));
      b->nsims = (int32_t)g.sims.size();
    }
    int32_t op = 0, ob = 0, os = 0, ot = 0;
    for (size_t k = 0; k < g.sims.size(); ++k) {
      le_sim* s = g.sims[k];
      const int cur = s->d.ctrl == s->ctrl_base ? 0 : 1;
      const Dev* dv = s->dev_dev + (cur ^ v);
      g.par[v].start[k] = op; g.bin[v].start[k] = ob; g.scan[v].start[k] = os; g.tile[v].start[k] = ot;
      g.one[v].start[k] = (int32_t)k;
      g.par[v].dev[k] = g.bin[v].dev[k] = g.scan[v].dev[k] = g.tile[v].dev[k] = g.one[v].dev[k] = dv;
      op += (s->d.n + kBlock - 1) / kBlock;
      ob += (s->d.n + kBinBlock - 1) / kBinBlock;
      os += s->d.sp_blocks;
      ot += s->d.ntiles;
    }
    const size_t m = g.sims.size();
    g.par[v].start[m] = op; g.bin[v].start[m] = ob; g.scan[v].start[m] = os; g.tile[v].start[m] = ot;
    g.one[v].start[m] = (int32_t)m;
  }
}

// Group the simulations (at most kMaxBatch per group).  LE_E_ARG for a null,
// repeated or foreign-stream simulation.
le_status plan_batch(le_sim* const* sims, int32_t nsims, std::vector<BatchGroup>& groups) {
  if (!sims || nsims < 1) return LE_E_ARG;
  for (int32_t a = 0; a < nsims; ++a) {
    if (!sims[a] || sims[a]->stream != sims[0]->stream) return LE_E_ARG;
    for (int32_t b = 0; b < a; ++b)
      if (sims[b] == sims[a]) return LE_E_ARG;
  }
  for (int32_t a = 0; a < nsims; ++a) {
    le_sim* s = sims[a];
    if (s->host_status) continue;  // latched: its kernels would be no-ops anyway
    BatchGroup* g = nullptr;
    for (BatchGroup& c : groups)
      if (c.sims.size() < (size_t)kMaxBatch && same_config(c.cfg, s->d)) { g = &c; break; }
    if (!g) {
      groups.emplace_back();
      g = &groups.back();
      g->cfg = s->d;
    }
    g->sims.push_back(s);
  }
  for (BatchGroup& g : groups) fill_group(g);
  return LE_OK;
}

le_status step_batch(std::vector<BatchGroup>& groups, hipStream_t q, int64_t nsteps, int32_t sample_every,
                     double* const* rings, int64_t ring_cap, le_sim* const* order, int32_t norder) {
  // ring of each member: the caller's rings are indexed like `order`
  auto ring_of = [&](le_sim* s) -> double* {
    for (int32_t k = 0; k < norder; ++k)
      if (order[k] == s) return rings[k];
    return nullptr;
  };
  int v = 0;  // which descriptor set is current
  le_status st = LE_OK;
  for (BatchGroup& g : groups)
    if (st == LE_OK) st = hip_check(launch_kick_drift_b(g.par[v], q));
  for (BatchGroup& g : groups)
    if (st == LE_OK) st = hip_check(launch_rebuild_b(g.bin[v], g.scan[v ^ 1], g.tile[v ^ 1], g.cfg, q));
  v ^= 1;
  int64_t ns = 0;
  for (int64_t k = 1; k <= nsteps && st == LE_OK; ++k) {
    const bool last = (k == nsteps);
    const bool sample = sample_every > 0 && (k % sample_every) == 0;
    for (BatchGroup& g : groups) {
      if (st != LE_OK) break;
      if (g.cfg.thermostat == LE_THERMO_DPD) {
        st = hip_check(launch_force_b(g.tile[v], g.par[v], g.cfg, q, kDpdForce, sample));
        if (st == LE_OK) st = hip_check(launch_integrate_b(g.tile[v], q, last, sample));
      } else {
        st = hip_check(launch_force_b(g.tile[v], g.par[v], g.cfg, q, last ? kStepLast : kStepFused, sample));
      }
      if (st == LE_OK && sample) {
        BatchOut out;
        memset(&out, 0, sizeof(out));
        for (size_t m = 0; m < g.sims.size(); ++m) out.ptr[m] = ring_of(g.sims[m]) + 6 * (ns % ring_cap);
        st = hip_check(launch_stress_final_b(g.one[v], out, q));
      }
    }
    if (sample) ++ns;
    if (st == LE_OK && !last) {
      for (BatchGroup& g : groups)
        if (st == LE_OK) st = hip_check(launch_rebuild_b(g.bin[v], g.scan[v ^ 1], g.tile[v ^ 1], g.cfg, q));
      v ^= 1;
    }
  }
  // every member's control copy alternated once per rebuild test (nsteps times)
  if (nsteps & 1)
    for (BatchGroup& g : groups)
      for (le_sim* s : g.sims) {
        const bool first = s->d.ctrl == s->ctrl_base;
        s->d.ctrl = first ? s->ctrl_base + 1 : s->ctrl_base;
        s->d.vmax = s->vmax_base + (first ? kSlots * kLineU64 : 0);
      }
  return st;
}

}  // namespace


namespace {

// Device address of `scratch` on the current device (looked up on the first
// call made with that device current).
le_status scratch_addr(void** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return LE_E_HIP;
  if (dev < 0 || dev >= kMaxDevices) return LE_E_HIP;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_addr[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return LE_E_HIP;
    g_scratch_addr[dev] = ptr;
  }
  *out = g_scratch_addr[dev];
  return LE_OK;
}

}  // namespace

extern "C" {

le_status le_workspace_bytes(const le_params* p, size_t* bytes) {
  if (!bytes) return LE_E_ARG;
  Geometry g;
  le_status st = validate(p, &g);
  if (st != LE_OK) return st;
  *bytes = carve(p, g, nullptr, nullptr, nullptr);
  return LE_OK;
}

le_status le_init(const le_params* p, const double* x0, const double* u0, const double* f0,
                  void* workspace, size_t ws_bytes, void* hip_stream, int64_t step0, le_sim** out) {
  if (!out || !x0 || !u0 || !workspace) return LE_E_ARG;
  *out = nullptr;
  Geometry g;
  le_status st = validate(p, &g);
  if (st != LE_OK) return st;
  size_t need = carve(p, g, nullptr, nullptr, nullptr);
  if (ws_bytes < need) return LE_E_WORKSPACE;
  le_sim* s = new (std::nothrow) le_sim();
  if (!s) return LE_E_ARG;
  s->host_status = 0;
  s->timing = 0;
  s->timing_stride = 1;
  s->tick = 0;
  s->ev_used = 0;
  for (int k = 0; k < 4; ++k) { s->phase_ms[k] = 0.0; s->phase_n[k] = 0; }
  s->p = *p;
  s->p.rc = g.rc;
  s->stream = (hipStream_t)hip_stream;
  char* base = (char*)(((uintptr_t)workspace + kAlign - 1) / kAlign * kAlign);
  carve(p, g, base, &s->d, s);
  fill_geometry(p, g, &s->d);
  double Delta0 = le_offset(step0, p->dt, s->d.sv, p->box[0]);
  st = hip_check(launch_load_state(s->d, s->stream, x0, u0, f0, step0, Delta0));
  if (st == LE_OK) {
    // the descriptors of batched launches: one per control copy
    Dev a = s->d, b = s->d;
    a.ctrl = s->ctrl_base; a.ctrl_other = s->ctrl_base + 1;
    a.vmax = s->vmax_base; a.vmax_other = s->vmax_base + kSlots * kLineU64;
    b.ctrl = a.ctrl_other; b.ctrl_other = a.ctrl;
    b.vmax = a.vmax_other; b.vmax_other = a.vmax;
    st = hip_check(launch_store_dev(a, b, s->dev_dev, s->stream));
  }
  if (st == LE_OK) st = rebuild(s, true, false);
  if (st == LE_OK && !f0)
    st = hip_check(launch_force(s->d, s->stream, s->d.thermostat == LE_THERMO_DPD ? kDpdForce : kInitForce,
                                false, nullptr, nullptr));
  if (st != LE_OK) {
    delete s;
    return st;
  }
  *out = s;
  return LE_OK;
}

le_status le_build_cells(le_sim* s, int32_t* cell_of, int32_t* order, int64_t* pairs,
                         int64_t pairs_cap, int64_t* n_pairs) {
  if (!s) return LE_E_ARG;
  if (s->host_status) return s->host_status;
  le_status st = rebuild(s, true, false);
  if (st == LE_OK && (cell_of || order))
    st = hip_check(launch_state_out(s->d, s->stream, nullptr, nullptr, cell_of, order));
  if (st == LE_OK && (pairs || n_pairs)) {
    st = hip_check(hipMemsetAsync(s->counter, 0, sizeof(unsigned long long), s->stream));
    if (st == LE_OK)
      st = hip_check(launch_pairs_out(s->d, s->stream, pairs, pairs ? pairs_cap : 0, s->counter));
    if (st == LE_OK && n_pairs) {
      unsigned long long cnt = 0;
      st = read_status(s);
      if (st == LE_OK && hipMemcpy(&cnt, s->counter, sizeof(cnt), hipMemcpyDeviceToHost) != hipSuccess)
        st = LE_E_HIP;
      *n_pairs = (int64_t)cnt;
    }
  }
  return st;
}

le_status le_forces(le_sim* s, double* f_out, double* virial6) {
  if (!s) return LE_E_ARG;
  if (s->host_status) return s->host_status;
  le_status st = hip_check(launch_force(s->d, s->stream, kForcesOnly, false, f_out, nullptr));
  if (st == LE_OK && virial6) st = hip_check(launch_stress_final(s->d, s->stream, virial6, true));
  return st;
}

le_status le_stress(le_sim* s, double* sigma6) {
  if (!s || !sigma6) return LE_E_ARG;
  if (s->host_status) return s->host_status;
  le_status st = hip_check(launch_force(s->d, s->stream, kForcesOnly, false, nullptr, nullptr));
  if (st == LE_OK) st = hip_check(launch_stress_final(s->d, s->stream, sigma6, false));
  return st;
}

le_status le_step(le_sim* s, int64_t nsteps, int32_t sample_every, double* stress_ring,
                  int64_t ring_cap) {
  if (!s || nsteps < 0) return LE_E_ARG;
  if (sample_every > 0 && (!stress_ring || ring_cap <= 0)) return LE_E_ARG;
  if (s->host_status) return s->host_status;
  if (nsteps == 0) return LE_OK;
  const Dev& d = s->d;
  hipStream_t q = s->stream;
  long ev = begin_phase(s, 2);
  le_status st = hip_check(launch_kick_drift(d, q));
  end_phase(s, ev);
  ev = begin_phase(s, 1);
  if (st == LE_OK) st = rebuild(s, false, true);
  end_phase(s, ev);
  int64_t ns = 0;
  for (int64_t k = 1; k <= nsteps && st == LE_OK; ++k) {
    const bool last = (k == nsteps);
    const bool sample = sample_every > 0 && (k % sample_every) == 0;
    // phase 0: the fused force kernel of plain steps, timed by the dispatch
    // itself; phase 3: sampled steps (force kernel with the virial, then the
    // stress reduction)
    if (d.thermostat == LE_THERMO_DPD) {
      // pair thermostat: all forces first, then the kicks and drift
      ev = sample ? begin_phase(s, 3) : -1;
      long ef = (!sample && s->tick++ % s->timing_stride == 0) ? reserve_pair(s, 0) : -1;
      st = hip_check(launch_force(d, q, kDpdForce, sample, nullptr, nullptr, ef >= 0 ? s->ev[2 * ef] : nullptr,
                                  ef >= 0 ? s->ev[2 * ef + 1] : nullptr));
      if (ef >= 0) s->ev_used = (size_t)ef + 1;
      if (st == LE_OK) st = hip_check(launch_integrate(d, q, last, sample));
      if (st == LE_OK && sample) {
        double* slot = stress_ring + 6 * (ns % ring_cap);
        ++ns;
        st = hip_check(launch_stress_final(d, q, slot, false));
      }
      end_phase(s, ev);
    } else if (sample) {
      ev = begin_phase(s, 3);
      st = hip_check(launch_force(d, q, last ? kStepLast : kStepFused, true, nullptr, nullptr));
      if (st == LE_OK) {
        double* slot = stress_ring + 6 * (ns % ring_cap);
        ++ns;
        st = hip_check(launch_stress_final(d, q, slot, false));
      }
      end_phase(s, ev);
    } else {
      ev = (s->tick++ % s->timing_stride == 0) ? reserve_pair(s, 0) : -1;
      st = hip_check(launch_force(d, q, last ? kStepLast : kStepFused, false, nullptr, nullptr,
                                  ev >= 0 ? s->ev[2 * ev] : nullptr,
                                  ev >= 0 ? s->ev[2 * ev + 1] : nullptr));
      if (ev >= 0) s->ev_used = (size_t)ev + 1;
    }
    if (st == LE_OK && !last) {
      ev = begin_phase(s, 1);
      st = rebuild(s, false, true);
      end_phase(s, ev);
    }
  }
  return st;
}

le_status le_step_batch(le_sim* const* sims, int32_t nsims, int64_t nsteps, int32_t sample_every,
                        double* const* stress_rings, int64_t ring_cap) {
  if (nsteps < 0) return LE_E_ARG;
  if (sample_every > 0 && (!stress_rings || ring_cap <= 0)) return LE_E_ARG;
  std::vector<BatchGroup> groups;
  le_status st = plan_batch(sims, nsims, groups);
  if (st != LE_OK) return st;
  if (sample_every > 0)
    for (int32_t k = 0; k < nsims; ++k)
      if (!stress_rings[k]) return LE_E_ARG;
  if (nsteps == 0 || groups.empty()) return LE_OK;
  return step_batch(groups, sims[0]->stream, nsteps, sample_every, stress_rings, ring_cap, sims, nsims);
}

le_status le_batch_graph_create(le_sim* const* sims, int32_t nsims, int64_t nsteps, int32_t sample_every,
                                double* const* stress_rings, int64_t ring_cap, le_graph** out) {
  if (!out || nsteps <= 0 || (nsteps & 1)) return LE_E_ARG;
  *out = nullptr;
  if (sample_every > 0 && (!stress_rings || ring_cap <= 0)) return LE_E_ARG;
  std::vector<BatchGroup> groups;
  le_status st = plan_batch(sims, nsims, groups);
  if (st != LE_OK) return st;
  if (groups.empty()) return LE_E_STATE;
  if (sample_every > 0)
    for (int32_t k = 0; k < nsims; ++k)
      if (!stress_rings[k]) return LE_E_ARG;
  hipStream_t q = sims[0]->stream;
  if (!q) return LE_E_STATE;  // the legacy default stream cannot be captured
  le_graph* g = new (std::nothrow) le_graph();
  if (!g) return LE_E_ARG;
  g->stream = q;
  for (BatchGroup& b : groups)
    for (le_sim* s : b.sims) {
      g->sims.push_back(s);
      g->ctrl_at.push_back(s->d.ctrl);
    }
  st = hip_check(hipStreamBeginCapture(q, hipStreamCaptureModeThreadLocal));
  if (st == LE_OK) {
    le_status st_step = step_batch(groups, q, nsteps, sample_every, stress_rings, ring_cap, sims, nsims);
    le_status st_end = hip_check(hipStreamEndCapture(q, &g->graph));
    st = st_step != LE_OK ? st_step : st_end;
  }
  for (size_t k = 0; k < g->sims.size() && st == LE_OK; ++k)
    if (g->sims[k]->d.ctrl != g->ctrl_at[k]) st = LE_E_STATE;  // cannot happen for even nsteps
  if (st == LE_OK) st = hip_check(hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0));
  if (st != LE_OK) {
    if (g->graph) (void)hipGraphDestroy(g->graph);
    delete g;
    return st;
  }
  *out = g;
  return LE_OK;
}

le_status le_observables(le_sim* s, int32_t nbins, double* out) {
  if (!s || !out || nbins < 1 || nbins > LE_MAX_BINS) return LE_E_ARG;
  if (s->host_status) return s->host_status;
  return hip_check(launch_observables(s->d, s->stream, nbins, out));
}

le_status le_unwrapped(le_sim* s, double* yz_out) {
  if (!s || !yz_out) return LE_E_ARG;
  if (s->host_status) return s->host_status;
  return hip_check(launch_unwrapped(s->d, s->stream, yz_out));
}

le_status le_msd(le_sim* s, const double* ref_yz, double* out2) {
  if (!s || !ref_yz || !out2) return LE_E_ARG;
  if (s->host_status) return s->host_status;
  return hip_check(launch_msd(s->d, s->stream, ref_yz, out2));
}

le_status le_get_state(le_sim* s, double* x, double* u, double* f, int64_t* step) {
  if (!s) return LE_E_ARG;
  if (s->host_status) return s->host_status;
  le_status st = rebuild(s, true, false);
  if (st == LE_OK && (x || u)) st = hip_check(launch_state_out(s->d, s->stream, x, u, nullptr, nullptr));
  if (st == LE_OK && f) {
    // the total force lives with the velocities; reuse the state scatter on it
    Dev tmp = s->d;
    tmp.vel[0] = s->d.frc[0];
    tmp.vel[1] = s->d.frc[1];
    st = hip_check(launch_state_out(tmp, s->stream, nullptr, f, nullptr, nullptr));
  }
  if (st == LE_OK) st = read_status(s);
  if (st == LE_OK && step) {
    if (hipMemcpy(step, &s->d.ctrl->step, sizeof(int64_t), hipMemcpyDeviceToHost) != hipSuccess)
      st = LE_E_HIP;
  }
  return st;
}

le_status le_graph_create(le_sim* s, int64_t nsteps, int32_t sample_every, double* stress_ring,
                          int64_t ring_cap, le_graph** out) {
  if (!s || !out || nsteps <= 0 || (nsteps & 1)) return LE_E_ARG;
  if (sample_every > 0 && (!stress_ring || ring_cap <= 0)) return LE_E_ARG;
  *out = nullptr;
  if (!s->stream) return LE_E_STATE;  // the legacy default stream cannot be captured
  if (s->host_status) return s->host_status;
  le_graph* g = new (std::nothrow) le_graph();
  if (!g) return LE_E_ARG;
  g->stream = s->stream;
  g->sims.push_back(s);
  g->ctrl_at.push_back(s->d.ctrl);
  const int32_t timing = s->timing;
  s->timing = 0;
  le_status st = hip_check(hipStreamBeginCapture(s->stream, hipStreamCaptureModeThreadLocal));
  if (st == LE_OK) {
    le_status st_step = le_step(s, nsteps, sample_every, stress_ring, ring_cap);
    le_status st_end = hip_check(hipStreamEndCapture(s->stream, &g->graph));
    st = st_step != LE_OK ? st_step : st_end;
  }
  s->timing = timing;
  if (st == LE_OK && s->d.ctrl != g->ctrl_at[0]) st = LE_E_STATE;  // cannot happen for even nsteps
  if (st == LE_OK) st = hip_check(hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0));
  if (st != LE_OK) {
    if (g->graph) (void)hipGraphDestroy(g->graph);
    delete g;
    return st;
  }
  *out = g;
  return LE_OK;
}

le_status le_graph_launch(le_graph* g) {
  if (!g) return LE_E_ARG;
  if (g->sims.size() == 1 && g->sims[0]->host_status) return g->sims[0]->host_status;
  for (size_t k = 0; k < g->sims.size(); ++k) {
    le_sim* s = g->sims[k];
    if (s->d.ctrl != g->ctrl_at[k]) {
      // an odd number of control updates since the capture: move the state to
      // the copy the graph reads (the simulation is unchanged)
      const bool first = g->ctrl_at[k] == s->ctrl_base;
      unsigned long long* vat = s->vmax_base + (first ? 0 : kSlots * kLineU64);
      le_status st = hip_check(launch_ctrl_copy(s->d.ctrl, g->ctrl_at[k], s->d.vmax, vat, s->stream));
      if (st != LE_OK) return st;
      s->d.ctrl = g->ctrl_at[k];
      s->d.vmax = vat;
    }
  }
  return hip_check(hipGraphLaunch(g->exec, g->stream));
}

le_status le_graph_destroy(le_graph* g) {
  if (!g) return LE_E_ARG;
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  delete g;
  return LE_OK;
}

le_status le_status_out(le_sim* s, int32_t* status_out) {
  if (!s || !status_out) return LE_E_ARG;
  return hip_check(launch_status_out(s->d, s->stream, status_out));
}

le_status le_sync(le_sim* s) {
  if (!s) return LE_E_ARG;
  return read_status(s);
}

le_status le_stats(le_sim* s, int64_t* rebuilds, int32_t* max_neighbors) {
  if (!s) return LE_E_ARG;
  le_status st = read_status(s);
  Ctrl c;
  Flags f;
  if (hipMemcpy(&c, s->d.ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost) != hipSuccess) return LE_E_HIP;
  if (hipMemcpy(&f, s->d.flags, sizeof(Flags), hipMemcpyDeviceToHost) != hipSuccess) return LE_E_HIP;
  if (rebuilds) *rebuilds = c.n_rebuilds;
  if (max_neighbors) {
    int32_t m = 0;
    for (int k = 0; k < kSlots; ++k) m = f.max_nb_slot[k * kLineInts] > m ? f.max_nb_slot[k * kLineInts] : m;
    *max_neighbors = m;
  }
  return st;
}

le_status le_timing_enable(le_sim* s, int32_t enabled) {
  if (!s) return LE_E_ARG;
  le_status st = fold_events(s);
  s->timing = enabled & 0xF;
  const int32_t stride = (enabled >> 8) & 0xFFFF;
  s->timing_stride = stride > 0 ? stride : 1;
  s->tick = 0;
  for (int k = 0; k < 4; ++k) { s->phase_ms[k] = 0.0; s->phase_n[k] = 0; }
  return st;
}

le_status le_timing_read(le_sim* s, double* ms, int64_t* launches) {
  if (!s) return LE_E_ARG;
  le_status st = fold_events(s);
  for (int k = 0; k < 4; ++k) {
    if (ms) ms[k] = s->phase_ms[k];
    if (launches) launches[k] = s->phase_n[k];
  }
  return st;
}

le_status le_destroy(le_sim* s) {
  if (!s) return LE_E_ARG;
  if (s->ev_used) (void)hipStreamSynchronize(s->stream);
  for (hipEvent_t e : s->ev) (void)hipEventDestroy(e);
  delete s;
  return LE_OK;
}

const char* le_strerror(le_status st) {
  switch (st) {
    case LE_OK: return "ok";
    case LE_E_ARG: return "invalid argument";
    case LE_E_GEOMETRY: return "box too small for the cutoff (need >= 3 cells of size >= rc+skin per axis)";
    case LE_E_WORKSPACE: return "workspace smaller than le_workspace_bytes()";
    case LE_E_BOND: return "FENE bond stretched to r >= R0";
    case LE_E_NONFINITE: return "non-finite position or velocity";
    case LE_E_CAPACITY: return "neighbour list or cell occupancy over capacity (raise max_neighbors, or lower the density)";
    case LE_E_HIP: return "HIP runtime error";
    case LE_E_STATE: return "call not valid in the current state";
    default: return "unknown status";
  }
}

le_status le_forces_static(const le_params* p, const double* x, double* f_out, double* virial6,
                           int32_t* status_out, int64_t step, void* hip_stream) {
  if (!p || !x || (!f_out && !virial6)) return LE_E_ARG;
  Geometry g;
  le_status st = validate(p, &g);
  if (st != LE_OK) return st;
  if (carve(p, g, nullptr, nullptr, nullptr) > kStaticScratchBytes) return LE_E_WORKSPACE;
  void* base = nullptr;
  st = scratch_addr(&base);
  if (st != LE_OK) return st;
  // a handle on the stack over the scratch (nothing on the heap): the same
  // launch sequence as le_init(x, u = 0) followed by le_forces
  le_sim s{};
  s.p = *p;
  s.p.rc = g.rc;
  s.stream = (hipStream_t)hip_stream;
  carve(p, g, (char*)base, &s.d, &s);
  fill_geometry(p, g, &s.d);
  const double Delta0 = le_offset(step, p->dt, s.d.sv, p->box[0]);
  st = hip_check(launch_load_state(s.d, s.stream, x, nullptr, nullptr, step, Delta0));
  if (st == LE_OK) st = rebuild(&s, true, false);
  if (st == LE_OK) st = hip_check(launch_force(s.d, s.stream, kForcesOnly, false, f_out, nullptr));
  if (st == LE_OK && virial6) st = hip_check(launch_stress_final(s.d, s.stream, virial6, true));
  if (st == LE_OK && status_out) st = hip_check(launch_status_out(s.d, s.stream, status_out));
  return st;
}

le_status le_offsets(double shear_rate, double Lx, double Ly, double dt, int64_t step0, int64_t count,
                     double* out, void* hip_stream) {
  if (!out || count < 0 || !(Lx > 0.0)) return LE_E_ARG;
  return hip_check(launch_offsets(shear_rate, Lx, Ly, dt, step0, count, out, (hipStream_t)hip_stream));
}

le_status le_philox(const uint32_t* ctr, const uint32_t* key, uint32_t* out, int64_t count,
                    void* hip_stream) {
  if (!ctr || !key || !out || count < 0) return LE_E_ARG;
  return hip_check(launch_philox(ctr, key, out, count, (hipStream_t)hip_stream));
}

}  // extern "C"
