// Batched stepping (lbm_batch_*): many domains of different sizes advance
// together.  Per step and per (lattice, storage, layout, collision) group there is one
// persistent launch of the multi-domain step kernel, which walks a tile table
// naming (domain, block of that domain); moving spheres of the group are then
// rebuilt by batched kernels that read their kinematics from a device table
// indexed by a device step counter.  The launches of two consecutive steps (and
// of sixteen) are captured once into HIP graphs and replayed; the tables live in device
// memory, so a new state parity or new kinematics only need new table
// contents, not a new graph.  The arithmetic per node is the single-domain
// kernel's, so results are bit-identical to lbm_step for any launch choice.
//
// Launch choices: grid (one workgroup per tile, or a persistent grid of k
// workgroups per compute unit) and tile order (call order; call order with each
// XCD given a contiguous share of the tiles; largest domain first with XCD
// shares).  The autotuner times each candidate on the batch itself and keeps the
// fastest per shape class (lattice, storage, layout, log2 of the tile count).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/lbm.h"
#include "error.hpp"
#include "internal.hpp"
#include "storage.hpp"

using namespace lbm;

namespace {

int bfail(int code, const std::string& msg) { return set_error(code, msg); }

#define BHIP(expr)                                                                                      \
  do {                                                                                                  \
    hipError_t e_ = (expr);                                                                             \
    if (e_ != hipSuccess) return bfail(LBM_EDEVICE, std::string(#expr ": ") + hipGetErrorString(e_));  \
  } while (0)

constexpr int KIN_ROWS = 256;        // steps of kinematics uploaded at a time
constexpr int LONG_PAIRS = 8;        // step pairs in the long graph (16 steps per replay)
constexpr int MAX_GROUP_DOMAINS = 1 << (32 - TILE_SHIFT);

struct Choice {
  int grid = 0;     // 0: one workgroup per tile; k > 0: k workgroups per compute unit
  int order = 1;    // 0 call order, 1 XCD shares, 2 largest first + XCD shares
};

// Device buffer that only grows.
struct DBuf {
  void* p = nullptr;
  size_t cap = 0;
};

struct Group {
  int lattice = 0, storage = 0;
  bool compact = false;
  bool trt = false;
  bool reg = false;                  // regularised wall non-equilibrium
  std::vector<int> members;          // indices into the batch's member list
  std::vector<int> movers;           // members with a moving sphere
  DBuf tab[2], tiles, mtab[2], waves;
  uint32_t nslots = 0, grid = 0, nwaves = 0;
  uint32_t ntiles = 0;
};

}  // namespace

struct lbm_batch_s {
  hipStream_t stream = nullptr;      // the members' stream
  hipStream_t cap = nullptr;         // private stream for graph capture
  int cus = 256;
  bool use_graph = true;
  bool autotune = false;
  Choice forced{-1, -1};             // set by options; -1 = tuned or default
  std::map<std::tuple<int, int, int, int, int, int>, Choice> tuned;
  std::map<std::tuple<int, int, int, int, int, int>, double> tuned_us;
  // composition
  std::vector<lbm_domain> members;
  std::vector<uint64_t> member_uid;  // identity of each member when the tables were built
  std::vector<int> cur_up;           // members' buffer parity the tables were written for
  std::vector<Group> groups;
  std::vector<Choice> group_choice;
  int nkin = 0;
  DBuf kin, ctr;
  // pinned staging and its last upload
  void* stage = nullptr;
  size_t stage_cap = 0;
  hipEvent_t stage_ev = nullptr;
  bool stage_pending = false;
  // graphs of one step pair and of LONG_PAIRS pairs
  hipGraphExec_t exec = nullptr;
  hipGraphExec_t exec_long = nullptr;
  std::vector<int64_t> sig;
  Choice last{-1, -1};
  double last_us = 0.0;
};

namespace {

int grow(DBuf& b, size_t bytes, lbm_batch_s* bt) {
  if (bytes <= b.cap) return LBM_OK;
  if (b.p) {
    BHIP(hipStreamSynchronize(bt->stream));
    (void)hipFree(b.p);
    b.p = nullptr;
    b.cap = 0;
  }
  const size_t cap = std::max<size_t>(bytes + bytes / 4, 256);
  hipError_t e = hipMalloc(&b.p, cap);
  if (e != hipSuccess) {
    b.p = nullptr;
    return bfail(e == hipErrorOutOfMemory ? LBM_ENOMEM : LBM_EDEVICE, std::string("hipMalloc: ") + hipGetErrorString(e));
  }
  b.cap = cap;
  return LBM_OK;
}

void drop(DBuf& b) {
  if (b.p) (void)hipFree(b.p);
  b.p = nullptr;
  b.cap = 0;
}

// Pinned staging area for table uploads; waits for the previous upload first.
int staging(lbm_batch_s* b, size_t bytes, char** out) {
  if (b->stage_pending) {
    BHIP(hipEventSynchronize(b->stage_ev));
    b->stage_pending = false;
  }
  if (bytes > b->stage_cap) {
    if (b->stage) (void)hipHostFree(b->stage);
    b->stage = nullptr;
    const size_t cap = std::max<size_t>(bytes + bytes / 4, 4096);
    BHIP(hipHostMalloc(&b->stage, cap, hipHostMallocDefault));
    b->stage_cap = cap;
  }
  *out = static_cast<char*>(b->stage);
  return LBM_OK;
}

// Copy pieces of the staging area to device buffers, in stream order.
struct Upload {
  const char* src;
  void* dst;
  size_t bytes;
};
int commit(lbm_batch_s* b, const std::vector<Upload>& ups) {
  for (const Upload& u : ups)
    if (u.bytes) BHIP(hipMemcpyAsync(u.dst, u.src, u.bytes, hipMemcpyHostToDevice, b->stream));
  BHIP(hipEventRecord(b->stage_ev, b->stream));
  b->stage_pending = true;
  return LBM_OK;
}

uint32_t blocks_of(const lbm_domain_s* d) { return (uint32_t)((d->g.nseg + WAVES_PER_BLOCK - 1) / WAVES_PER_BLOCK); }

std::tuple<int, int, int, int, int, int> shape_key(const Group& g) {
  int lg = 0;
  while ((1u << (lg + 1)) <= std::max<uint32_t>(g.ntiles, 1)) ++lg;
  return {g.lattice, g.storage, g.compact ? 1 : 0, g.trt ? 1 : 0, g.reg ? 1 : 0, lg};
}

// Tile table of a group for one launch choice (see the kernel's comment).
std::vector<uint32_t> tile_table(const lbm_batch_s* b, const Group& g, const Choice& ch, uint32_t* grid) {
  std::vector<int> order(g.members.size());
  for (size_t k = 0; k < order.size(); ++k) order[k] = (int)k;
  if (ch.order == 2)
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
      return blocks_of(b->members[g.members[x]]) > blocks_of(b->members[g.members[y]]);
    });
  std::vector<uint32_t> nat;
  nat.reserve(g.ntiles);
  for (int k : order) {
    const uint32_t nb = blocks_of(b->members[g.members[k]]);
    for (uint32_t t = 0; t < nb; ++t) nat.push_back(((uint32_t)k << TILE_SHIFT) | t);
  }
  const uint32_t n = (uint32_t)nat.size();
  const uint32_t n8 = (n + 7) / 8 * 8;
  uint32_t G = n8;
  if (ch.grid > 0) G = std::min<uint32_t>(n8, (uint32_t)(ch.grid * b->cus) / 8 * 8);
  if (G == 0) G = 8;
  const uint32_t S = (n + G - 1) / G * G;
  std::vector<uint32_t> tab(S, TILE_EMPTY);
  if (ch.order == 0) {
    for (uint32_t s = 0; s < n; ++s) tab[s] = nat[s];
  } else {
    // XCD k (workgroups k, k + 8, ...) takes the k-th contiguous eighth of the tiles
    uint32_t start = 0;
    for (uint32_t k = 0; k < 8; ++k) {
      const uint32_t size = n / 8 + (k < n % 8 ? 1u : 0u);
      for (uint32_t m = 0; m < size; ++m) tab[k + 8 * m] = nat[start + m];
      start += size;
    }
  }
  *grid = G;
  return tab;
}

Choice choice_for(const lbm_batch_s* b, const Group& g) {
  Choice c;
  auto it = b->tuned.find(shape_key(g));
  if (it != b->tuned.end()) c = it->second;
  if (b->forced.grid >= 0) c.grid = b->forced.grid;
  if (b->forced.order >= 0) c.order = b->forced.order;
  return c;
}

// Write the step and moving tables of every group for the members' current
// parity and the given choices, upload them, and return the launch signature.
int write_tables(lbm_batch_s* b) {
  size_t bytes = 0;
  std::vector<std::vector<uint32_t>> tiles(b->groups.size());
  std::vector<std::vector<uint32_t>> waves(b->groups.size());
  for (size_t gi = 0; gi < b->groups.size(); ++gi) {
    Group& g = b->groups[gi];
    tiles[gi] = tile_table(b, g, b->group_choice[gi], &g.grid);
    g.nslots = (uint32_t)tiles[gi].size();
    for (size_t m = 0; m < g.movers.size(); ++m) {
      const lbm_domain_s* d = b->members[g.members[g.movers[m]]];
      for (int64_t w = 0; w < d->nreg; ++w) waves[gi].push_back(((uint32_t)m << TILE_SHIFT) | (uint32_t)w);
    }
    g.nwaves = (uint32_t)waves[gi].size();
    bytes += 2 * g.members.size() * sizeof(StepParams) + tiles[gi].size() * 4 + 2 * g.movers.size() * sizeof(MovingParams) +
             waves[gi].size() * 4 + 64 * 6;
  }
  for (size_t gi = 0; gi < b->groups.size(); ++gi) {
    Group& g = b->groups[gi];
    for (int p = 0; p < 2; ++p) {
      if (int e = grow(g.tab[p], g.members.size() * sizeof(StepParams), b)) return e;
      if (int e = grow(g.mtab[p], std::max<size_t>(1, g.movers.size()) * sizeof(MovingParams), b)) return e;
    }
    if (int e = grow(g.tiles, tiles[gi].size() * 4, b)) return e;
    if (int e = grow(g.waves, std::max<size_t>(1, waves[gi].size()) * 4, b)) return e;
  }
  char* st = nullptr;
  if (int e = staging(b, bytes, &st)) return e;
  std::vector<Upload> ups;
  size_t off = 0;
  auto put = [&](const void* src, size_t n, void* dst) {
    std::memcpy(st + off, src, n);
    ups.push_back({st + off, dst, n});
    off += (n + 63) / 64 * 64;
  };
  int kin_slot = 0;
  for (size_t gi = 0; gi < b->groups.size(); ++gi) {
    Group& g = b->groups[gi];
    for (int p = 0; p < 2; ++p) {
      std::vector<StepParams> sp;
      for (int mi : g.members) {
        const lbm_domain_s* d = b->members[mi];
        sp.push_back(step_params(d, d->cur ^ p));
      }
      put(sp.data(), sp.size() * sizeof(StepParams), g.tab[p].p);
      std::vector<MovingParams> mp;
      int slot = kin_slot;
      for (int m : g.movers) {
        const lbm_domain_s* d = b->members[g.members[m]];
        MovingParams q = moving_params(d, d->cur ^ p ^ 1);   // refill the state the step wrote
        q.kin_slot = slot++;
        mp.push_back(q);
      }
      if (!mp.empty()) put(mp.data(), mp.size() * sizeof(MovingParams), g.mtab[p].p);
    }
    kin_slot += (int)g.movers.size();
    put(tiles[gi].data(), tiles[gi].size() * 4, g.tiles.p);
    if (!waves[gi].empty()) put(waves[gi].data(), waves[gi].size() * 4, g.waves.p);
  }
  b->nkin = kin_slot;
  if (b->nkin > 0) {
    if (int e = grow(b->kin, (size_t)KIN_ROWS * b->nkin * sizeof(MovingKin), b)) return e;
    if (int e = grow(b->ctr, 8, b)) return e;
  }
  if (int e = commit(b, ups)) return e;
  b->cur_up.clear();
  for (lbm_domain d : b->members) b->cur_up.push_back(d->cur);
  return LBM_OK;
}

std::vector<int64_t> launch_signature(const lbm_batch_s* b) {
  std::vector<int64_t> s;
  for (const Group& g : b->groups) {
    for (int64_t v : {(int64_t)g.lattice, (int64_t)g.storage, (int64_t)g.compact, (int64_t)g.trt, (int64_t)g.reg,
                      (int64_t)(intptr_t)g.tab[0].p,
                      (int64_t)(intptr_t)g.tab[1].p, (int64_t)(intptr_t)g.tiles.p, (int64_t)g.nslots, (int64_t)g.grid,
                      (int64_t)g.movers.size(), (int64_t)(intptr_t)g.mtab[0].p, (int64_t)(intptr_t)g.mtab[1].p,
                      (int64_t)(intptr_t)g.waves.p, (int64_t)g.nwaves})
      s.push_back(v);
  }
  s.push_back((int64_t)(intptr_t)b->kin.p);
  s.push_back((int64_t)(intptr_t)b->ctr.p);
  s.push_back(b->nkin);
  return s;
}

// Launches of one step; p = 0: the members' states are in the buffers the
// tables were written for, p = 1: in the other ones.
hipError_t enqueue_step(lbm_batch_s* b, int p, hipStream_t s) {
  for (const Group& g : b->groups) {
    hipError_t e = launch_step_batch(g.lattice, g.storage, g.compact, g.trt, g.reg, static_cast<const StepParams*>(g.tab[p].p),
                                     static_cast<const uint32_t*>(g.tiles.p), g.nslots, g.grid, s);
    if (e != hipSuccess) return e;
  }
  bool any = false;
  for (const Group& g : b->groups) {
    if (g.movers.empty()) continue;
    any = true;
    MovingBatch mb{};
    mb.tab = static_cast<const MovingParams*>(g.mtab[p].p);
    mb.nbox = (int32_t)g.movers.size();
    for (int m : g.movers) mb.multi |= b->members[g.members[m]]->mv_ns > 1 ? 1 : 0;
    mb.waves = static_cast<const uint32_t*>(g.waves.p);
    mb.nwaves = g.nwaves;
    mb.kin = static_cast<const MovingKin*>(b->kin.p);
    mb.nkin = b->nkin;
    mb.ctr = static_cast<const int64_t*>(b->ctr.p);
    hipError_t e = launch_moving_batch(g.lattice, storage_format(g.storage), mb, s);
    if (e != hipSuccess) return e;
  }
  if (any) return launch_advance(static_cast<int64_t*>(b->ctr.p), s);
  return hipSuccess;
}

int capture_pairs(lbm_batch_s* b, int pairs, hipGraphExec_t* out) {
  hipGraph_t graph = nullptr;
  BHIP(hipStreamBeginCapture(b->cap, hipStreamCaptureModeRelaxed));
  hipError_t e = hipSuccess;
  for (int k = 0; k < pairs && e == hipSuccess; ++k) {
    e = enqueue_step(b, 0, b->cap);
    if (e == hipSuccess) e = enqueue_step(b, 1, b->cap);
  }
  hipError_t e2 = hipStreamEndCapture(b->cap, &graph);
  if (e != hipSuccess || e2 != hipSuccess) {
    if (graph) (void)hipGraphDestroy(graph);
    return bfail(LBM_EDEVICE, std::string("graph capture: ") + hipGetErrorString(e != hipSuccess ? e : e2));
  }
  e = hipGraphInstantiate(out, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e != hipSuccess) {
    *out = nullptr;
    return bfail(LBM_EDEVICE, std::string("graph instantiate: ") + hipGetErrorString(e));
  }
  return LBM_OK;
}

void destroy_graphs(lbm_batch_s* b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->exec_long) (void)hipGraphExecDestroy(b->exec_long);
  b->exec = b->exec_long = nullptr;
}

int capture(lbm_batch_s* b) {
  if (b->exec || b->exec_long) {
    BHIP(hipStreamSynchronize(b->stream));   // no replay of the old graphs in flight
    destroy_graphs(b);
  }
  if (int e = capture_pairs(b, 1, &b->exec)) return e;
  if (int e = capture_pairs(b, LONG_PAIRS, &b->exec_long)) {
    destroy_graphs(b);
    return e;
  }
  b->sig = launch_signature(b);
  return LBM_OK;
}

void release_groups(lbm_batch_s* b) {
  destroy_graphs(b);
  for (Group& g : b->groups) {
    drop(g.tab[0]);
    drop(g.tab[1]);
    drop(g.tiles);
    drop(g.mtab[0]);
    drop(g.mtab[1]);
    drop(g.waves);
  }
  b->groups.clear();
  b->cur_up.clear();
  b->members.clear();
  b->member_uid.clear();
}

// Set the membership: group the domains, pick each group's launch choice and
// write the tables when anything changed.
int prepare(lbm_batch_s* b, const lbm_domain* ds, int32_t n) {
  // a domain is the same member only if both its address and its uid match:
  // a new domain can be allocated at a freed one's address
  bool same = (int32_t)b->members.size() == n && b->member_uid.size() == b->members.size();
  for (int32_t k = 0; same && k < n; ++k) same = b->members[k] == ds[k] && b->member_uid[k] == ds[k]->uid;
  if (!same) {
    if (!b->groups.empty()) {   // pending launches may still read the old tables
      BHIP(hipStreamSynchronize(b->stream));
      release_groups(b);
    }
    b->members.assign(ds, ds + n);
    b->member_uid.clear();
    for (int32_t k = 0; k < n; ++k) b->member_uid.push_back(ds[k]->uid);
    for (int32_t k = 0; k < n; ++k) {
      const lbm_domain_s* d = ds[k];
      Group* g = nullptr;
      const bool trt = d->desc.collision == LBM_TRT;
      const bool reg = d->wall_neq == LBM_NEQ_REGULARIZED;
      for (Group& x : b->groups)
        if (x.lattice == d->desc.lattice && x.storage == d->skind && x.compact == (d->g.compact != 0) &&
            x.trt == trt && x.reg == reg)
          g = &x;
      if (!g) {
        b->groups.emplace_back();
        g = &b->groups.back();
        g->lattice = d->desc.lattice;
        g->storage = d->skind;
        g->compact = d->g.compact != 0;
        g->trt = trt;
        g->reg = reg;
      }
      if ((int)g->members.size() >= MAX_GROUP_DOMAINS) return bfail(LBM_EINVAL, "too many domains of one kind in a batch");
      if (d->moving) g->movers.push_back((int)g->members.size());
      g->members.push_back(k);
      g->ntiles += blocks_of(d);
    }
    b->group_choice.clear();
  }
  std::vector<Choice> want;
  for (const Group& g : b->groups) want.push_back(choice_for(b, g));
  bool same_choice = b->group_choice.size() == want.size();
  for (size_t k = 0; same_choice && k < want.size(); ++k)
    same_choice = want[k].grid == b->group_choice[k].grid && want[k].order == b->group_choice[k].order;
  bool same_parity = same && same_choice && b->cur_up.size() == b->members.size();
  for (size_t k = 0; same_parity && k < b->members.size(); ++k) same_parity = b->cur_up[k] == b->members[k]->cur;
  if (!same_parity) {
    b->group_choice = want;
    if (int e = write_tables(b)) return e;
  }
  return LBM_OK;
}

// Upload kinematics rows for the next `rows` steps and reset the step counter.
int upload_kin(lbm_batch_s* b, int64_t done, int rows) {
  if (b->nkin == 0) return LBM_OK;
  char* st = nullptr;
  const size_t kb = (size_t)rows * b->nkin * sizeof(MovingKin);
  if (int e = staging(b, kb + 64, &st)) return e;
  MovingKin* k = reinterpret_cast<MovingKin*>(st);
  int slot = 0;
  for (const Group& g : b->groups)
    for (int m : g.movers) {
      const lbm_domain_s* d = b->members[g.members[m]];
      for (int r = 0; r < rows; ++r) k[(size_t)r * b->nkin + slot] = moving_kin(d, d->steps + done + r + 1);
      ++slot;
    }
  int64_t* zero = reinterpret_cast<int64_t*>(st + (kb + 63) / 64 * 64);
  *zero = 0;
  return commit(b, {{st, b->kin.p, kb}, {reinterpret_cast<const char*>(zero), b->ctr.p, 8}});
}

// Advance every member by n steps with the current tables.
int run(lbm_batch_s* b, int32_t n, bool graph) {
  if (n <= 0) return LBM_OK;
  if (graph && (!b->exec || b->sig != launch_signature(b)))
    if (int e = capture(b)) return e;
  int64_t done = 0;
  while (done < n) {
    const int rows = (int)std::min<int64_t>(n - done, KIN_ROWS);
    if (int e = upload_kin(b, done, rows)) return e;
    int r = 0;
    if (graph) {
      for (; r + 2 * LONG_PAIRS <= rows; r += 2 * LONG_PAIRS) BHIP(hipGraphLaunch(b->exec_long, b->stream));
      for (; r + 1 < rows; r += 2) BHIP(hipGraphLaunch(b->exec, b->stream));
    }
    for (; r < rows; ++r) BHIP(enqueue_step(b, r & 1, b->stream));
    done += rows;
  }
  for (lbm_domain d : b->members) {
    d->cur ^= (n & 1);
    d->steps += n;
  }
  return LBM_OK;
}

int check_members(lbm_batch_s* b, const lbm_domain* ds, int32_t n) {
  if (!ds && n > 0) return bfail(LBM_EINVAL, "null domain list");
  if (n < 0) return bfail(LBM_EINVAL, "n < 0");
  std::vector<lbm_domain> seen(ds, ds + n);
  std::sort(seen.begin(), seen.end());
  for (int32_t k = 0; k < n; ++k) {
    if (!ds[k]) return bfail(LBM_EINVAL, "null domain at position " + std::to_string(k));
    if (!ds[k]->links_ok) return bfail(LBM_ESTATE, "domain " + std::to_string(k) + ": boundary links not set");
    if (ds[k]->stream != b->stream) return bfail(LBM_EINVAL, "domain " + std::to_string(k) + " uses another stream than the batch");
    if (blocks_of(ds[k]) > TILE_MASK + 1u) return bfail(LBM_EINVAL, "domain " + std::to_string(k) + " too large for a batch");
  }
  if (std::adjacent_find(seen.begin(), seen.end()) != seen.end()) return bfail(LBM_EINVAL, "a domain appears twice");
  return LBM_OK;
}

}  // namespace

extern "C" {

int lbm_batch_create(void* stream, lbm_batch* out) {
  if (!out) return bfail(LBM_EINVAL, "null argument");
  lbm_batch_s* b = new lbm_batch_s();
  b->stream = static_cast<hipStream_t>(stream);
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&b->cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&b->stage_ev, hipEventDisableTiming);
  if (e != hipSuccess) {
    if (b->cap) (void)hipStreamDestroy(b->cap);
    delete b;
    return bfail(LBM_EDEVICE, std::string("lbm_batch_create: ") + hipGetErrorString(e));
  }
  *out = b;
  clear_error();
  return LBM_OK;
}

int lbm_batch_set_option(lbm_batch b, int32_t option, int32_t value) {
  if (!b) return bfail(LBM_EINVAL, "null batch");
  switch (option) {
    case LBM_BATCH_GRAPH:
      if (value != 0 && value != 1) break;
      b->use_graph = value != 0;
      return LBM_OK;
    case LBM_BATCH_GRID:
      if (value < -1 || value > 64) break;
      b->forced.grid = value;
      return LBM_OK;
    case LBM_BATCH_ORDER:
      if (value < -1 || value > 2) break;
      b->forced.order = value;
      return LBM_OK;
    case LBM_BATCH_AUTOTUNE:
      if (value != 0 && value != 1) break;
      b->autotune = value != 0;
      return LBM_OK;
    default:
      break;
  }
  return bfail(LBM_EINVAL, "invalid batch option or value");
}

int lbm_batch_autotune(lbm_batch b, const lbm_domain* ds, int32_t n, int32_t steps_per_candidate) {
  if (!b) return bfail(LBM_EINVAL, "null batch");
  if (int e = check_members(b, ds, n)) return e;
  if (steps_per_candidate < 1) return bfail(LBM_EINVAL, "steps_per_candidate < 1");
  if (n == 0) return LBM_OK;
  const Choice saved = b->forced;
  static const int grids[] = {0, 2, 4, 6};
  static const int orders[] = {0, 1, 2};
  hipEvent_t e0 = nullptr, e1 = nullptr;
  BHIP(hipEventCreate(&e0));
  BHIP(hipEventCreate(&e1));
  int rc = LBM_OK;
  double best = 1e300;
  Choice bc;
  // one warm-up pass so that every candidate runs on warm caches and code
  b->forced = Choice{0, 1};
  rc = prepare(b, ds, n);
  if (rc == LBM_OK) rc = run(b, n > 0 ? 1 : 0, false);
  for (int gsel : grids) {
    for (int osel : orders) {
      if (rc != LBM_OK) break;
      b->forced = Choice{gsel, osel};
      rc = prepare(b, ds, n);
      if (rc != LBM_OK) break;
      hipError_t e = hipEventRecord(e0, b->stream);
      if (e == hipSuccess) rc = run(b, steps_per_candidate, false);
      if (e == hipSuccess && rc == LBM_OK) e = hipEventRecord(e1, b->stream);
      if (e == hipSuccess && rc == LBM_OK) e = hipEventSynchronize(e1);
      float ms = 0.f;
      if (e == hipSuccess && rc == LBM_OK) e = hipEventElapsedTime(&ms, e0, e1);
      if (e != hipSuccess) rc = bfail(LBM_EDEVICE, std::string("autotune: ") + hipGetErrorString(e));
      if (rc != LBM_OK) break;
      const double us = 1e3 * ms / steps_per_candidate;
      if (us < best) {
        best = us;
        bc = b->forced;
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  b->forced = saved;
  if (rc != LBM_OK) return rc;
  for (const Group& g : b->groups) {
    b->tuned[shape_key(g)] = bc;
    b->tuned_us[shape_key(g)] = best;
  }
  b->last = bc;
  b->last_us = best;
  clear_error();
  return LBM_OK;
}

int lbm_batch_step(lbm_batch b, const lbm_domain* ds, int32_t n, int32_t n_steps) {
  if (!b) return bfail(LBM_EINVAL, "null batch");
  if (int e = check_members(b, ds, n)) return e;
  if (n_steps < 0) return bfail(LBM_EINVAL, "n_steps < 0");
  if (n == 0 || n_steps == 0) return LBM_OK;
  for (int32_t k = 0; k < n; ++k)
    if (n_steps > path_steps_left(ds[k]))
      return bfail(LBM_ESTATE, "domain " + std::to_string(k) + ": the sphere's path ends after " +
                                   std::to_string(path_steps_left(ds[k])) + " more steps");
  if (int e = prepare(b, ds, n)) return e;
  if (b->autotune) {
    bool known = true;
    for (const Group& g : b->groups) known = known && b->tuned.count(shape_key(g));
    const int32_t spc = 4, need = 1 + 12 * spc;
    if (!known && n_steps >= need) {
      if (int e = lbm_batch_autotune(b, ds, n, spc)) return e;
      n_steps -= need;
      if (int e = prepare(b, ds, n)) return e;
    }
  }
  if (int e = run(b, n_steps, b->use_graph)) return e;
  clear_error();
  return LBM_OK;
}

int lbm_batch_get_choice(lbm_batch b, int32_t* grid, int32_t* order, double* us_per_step) {
  if (!b) return bfail(LBM_EINVAL, "null batch");
  Choice c = b->groups.empty() ? Choice{} : b->group_choice.empty() ? Choice{} : b->group_choice[0];
  if (grid) *grid = c.grid;
  if (order) *order = c.order;
  if (us_per_step) *us_per_step = b->last_us;
  return LBM_OK;
}

int lbm_batch_free(lbm_batch b) {
  if (!b) return bfail(LBM_EINVAL, "null batch");
  (void)hipStreamSynchronize(b->stream);
  release_groups(b);
  drop(b->kin);
  drop(b->ctr);
  if (b->stage) (void)hipHostFree(b->stage);
  if (b->stage_ev) (void)hipEventDestroy(b->stage_ev);
  if (b->cap) (void)hipStreamDestroy(b->cap);
  delete b;
  return LBM_OK;
}

int lbm_step_batch(const lbm_domain* ds, int32_t n, int32_t n_steps) {
  if (n < 0 || (n > 0 && (!ds || !ds[0]))) return bfail(LBM_EINVAL, "invalid domain list");
  if (n == 0) return LBM_OK;
  lbm_batch b = nullptr;
  if (int e = lbm_batch_create(ds[0]->stream, &b)) return e;
  lbm_batch_set_option(b, LBM_BATCH_GRAPH, 0);
  int rc = lbm_batch_step(b, ds, n, n_steps);
  const std::string msg = lbm_last_error();
  lbm_batch_free(b);
  if (rc != LBM_OK) return bfail(rc, msg);
  return LBM_OK;
}

}  // extern "C"
