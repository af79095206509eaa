// lbm_api.cpp -- host side of the C interface declared in include/lbm0d3d.h.
//
// Validates geometry and parameters, lays out the caller's device buffers,
// builds the per-instance tables the kernels read (block -> instance,
// boundary-layer cell lists, reduction work table, wall band), enqueues the
// kernels of every step on the caller's stream (eagerly or from a captured
// HIP graph of one even + one odd step) and converts populations between the
// storage precision and host FP64 for read-back.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/lbm0d3d.h"
#include "lbm_internal.h"

using namespace lbm;

namespace {

constexpr int EXh[NQ] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
constexpr int EYh[NQ] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
constexpr int EZh[NQ] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
constexpr int NTIMED = 5;   // kinds of timed launches (lbm_kernel_time ids)
constexpr int OPPh[NQ] = {0, 2, 1, 4, 3, 6, 5, 8, 7, 10, 9, 12, 11, 14, 13, 16, 15, 18, 17};
constexpr double W[NQ] = {1.0 / 3,  1.0 / 18, 1.0 / 18, 1.0 / 18, 1.0 / 18, 1.0 / 18, 1.0 / 18,
                          1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36,
                          1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

int elem_size(int prec) { return prec == 0 ? 8 : (prec == 1 ? 4 : 2); }
int r4_size(int prec) { return prec == 0 ? 32 : 16; }

// -------- host conversions to and from the storage precision --------------
uint16_t f32_to_bf16_rne(float f) {
  uint32_t u;
  std::memcpy(&u, &f, 4);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
float bf16_to_f32(uint16_t h) {
  uint32_t u = (uint32_t)h << 16;
  float f;
  std::memcpy(&f, &u, 4);
  return f;
}
uint16_t f32_to_f16_rne(float f) {
  _Float16 h = (_Float16)f;
  uint16_t u;
  std::memcpy(&u, &h, 2);
  return u;
}
float f16_to_f32(uint16_t u) {
  _Float16 h;
  std::memcpy(&h, &u, 2);
  return (float)h;
}

struct Geometry {
  int nx, ny, nz;
  int64_t ncell;
  std::vector<uint8_t> flags;        // with F_NEAR (and F_BAND) bits
  std::vector<uint64_t> nbr;         // NEAR cells: the 18 neighbour types, 3 bits each
  std::vector<int32_t> lay[NPL];   // boundary layers: inlet, outlet 0, mid-length, outlets 1..7
  // FLUID cells next to a 0D-coupled ghost (within one cell in each axis),
  // ascending: where the normal-neighbour extrapolation does its work
  std::vector<int32_t> ghost_near;
};

// Checks the cell types and derives the NEAR bits, the neighbour-type words
// of NEAR cells and the boundary-layer lists.
bool build_geometry(const lbm_config& c, Geometry& g, std::string& err) {
  if (c.nx < 3 || c.ny < 3 || c.nz < 3) { err = "box dimensions must be >= 3"; return false; }
  if (!(c.tau > 0.5)) { err = "tau must be > 0.5"; return false; }
  if (c.nee_variant != 0 && c.nee_variant != 1) { err = "nee_variant must be 0 or 1"; return false; }
  if (!c.flags) { err = "flags is NULL"; return false; }
  g.nx = c.nx; g.ny = c.ny; g.nz = c.nz;
  g.ncell = (int64_t)c.nx * c.ny * c.nz;
  if (g.ncell > (int64_t)1 << 31) { err = "instance too large"; return false; }
  g.flags.assign(c.flags, c.flags + g.ncell);
  auto at = [&](int x, int y, int z) -> uint8_t& { return g.flags[x + (int64_t)g.nx * (y + (int64_t)g.ny * z)]; };
  for (int z = 0; z < g.nz; ++z)
    for (int y = 0; y < g.ny; ++y)
      for (int x = 0; x < g.nx; ++x) {
        const uint8_t raw = at(x, y, z), t = raw & TYPE_MASK;
        const bool face = x == 0 || y == 0 || z == 0 || x == g.nx - 1 || y == g.ny - 1 || z == g.nz - 1;
        if (t > T_EXTP || (raw & (F_NEAR | F_BAND)) || (t != T_OUTLET && (raw >> OUT_SHIFT)))
          { err = "cell type out of range (only OUTLET ghosts carry an outlet index in bits 5-7)"; return false; }
        if (face && t == T_FLUID) { err = "FLUID cell on the box boundary"; return false; }
        if (t == T_INLET && z != 0) { err = "INLET cell off the plane z = 0"; return false; }
        if (t == T_OUTLET && z != g.nz - 1) { err = "OUTLET cell off the plane z = nz-1"; return false; }
        if (t == T_EXTP && !face) { err = "EXTP cell inside the box"; return false; }
      }
  g.nbr.assign(g.ncell, 0);
  for (int z = 1; z < g.nz - 1; ++z)
    for (int y = 1; y < g.ny - 1; ++y)
      for (int x = 1; x < g.nx - 1; ++x) {
        uint8_t& t = at(x, y, z);
        if (t != T_FLUID) continue;
        uint64_t w = 0;
        for (int i = 1; i < NQ; ++i)   // source of direction i: c - e_i (type bits only)
          w |= (uint64_t)(at(x - EXh[i], y - EYh[i], z - EZh[i]) & TYPE_MASK) << (3 * i);
        if (w != 0) {
          t |= F_NEAR;
          g.nbr[x + (int64_t)g.nx * (y + (int64_t)g.ny * z)] = w;
        }
      }
  // inlet layer (plane 0) and the layer of each outlet k (plane
  // outlet_slot(k)): FLUID cells of z = 1 / z = nz-2 next to the ghost plane
  for (int pl = 0; pl < NPL; ++pl) g.lay[pl].clear();
  for (int side = 0; side < 1 + NOUT; ++side) {
    const int zl = side == 0 ? 1 : g.nz - 2, zg = side == 0 ? 0 : g.nz - 1;
    const uint8_t gt = side == 0 ? T_INLET : T_OUTLET;
    const int pl = side == 0 ? 0 : outlet_slot(side - 1);
    for (int y = 0; y < g.ny; ++y)
      for (int x = 0; x < g.nx; ++x) {
        const uint8_t gc = at(x, y, zg);
        if ((at(x, y, zl) & TYPE_MASK) == T_FLUID && (gc & TYPE_MASK) == gt &&
            (side == 0 || (gc >> OUT_SHIFT) == side - 1))
          g.lay[pl].push_back(x + g.nx * (y + g.ny * zl));
      }
  }
  g.ghost_near.clear();
  if (c.nee_variant == 1) {
    std::vector<uint8_t> mark(g.ncell, 0);
    for (int z = 0; z < g.nz; ++z)
      for (int y = 0; y < g.ny; ++y)
        for (int x = 0; x < g.nx; ++x) {
          const uint8_t t = at(x, y, z) & TYPE_MASK;
          if (t != T_INLET && t != T_OUTLET && t != T_EXTP) continue;
          for (int dz = -1; dz <= 1; ++dz)
            for (int dy = -1; dy <= 1; ++dy)
              for (int dx = -1; dx <= 1; ++dx) {
                const int xx = x + dx, yy = y + dy, zz = z + dz;
                if (xx < 0 || yy < 0 || zz < 0 || xx >= g.nx || yy >= g.ny || zz >= g.nz) continue;
                if ((at(xx, yy, zz) & TYPE_MASK) == T_FLUID) mark[xx + (int64_t)g.nx * (yy + (int64_t)g.ny * zz)] = 1;
              }
        }
    for (int64_t cell = 0; cell < g.ncell; ++cell)
      if (mark[cell]) g.ghost_near.push_back((int32_t)cell);
  }
  // mid-length plane z = nz/2, over the columns of the inlet's lumen (cells
  // above an INLET ghost): its flux and pressure are recorded, not coupled
  g.lay[2].clear();
  for (int y = 0; y < g.ny; ++y)
    for (int x = 0; x < g.nx; ++x)
      if ((at(x, y, g.nz / 2) & TYPE_MASK) == T_FLUID && (at(x, y, 0) & TYPE_MASK) == T_INLET)
        g.lay[2].push_back(x + g.nx * (y + g.ny * (g.nz / 2)));
  return true;
}

struct Layout {
  size_t flags, nbr, inst, ctab, btab, lay, red, red_part, bc, st, wave, owave, v0, err, moved, walls, cwalls;
  size_t bmark, btmp, bcnt, gate, total;
  int64_t NT, nbcnt;
  int ntile_max, nred, nlay, wave_cap;
  int64_t nv0;
};

void plan(const std::vector<Geometry>& G, int prec, int wave_cap, Layout& L, std::vector<InstDesc>* inst,
          std::vector<int32_t>* lay, std::vector<RedTab>* red) {
  L.NT = 0; L.ntile_max = 0; L.nred = 0; L.nlay = 0; L.nv0 = 0; L.wave_cap = wave_cap; L.nbcnt = 0;
  for (size_t k = 0; k < G.size(); ++k) {
    const Geometry& g = G[k];
    InstDesc d;
    std::memset(&d, 0, sizeof d);
    d.nx = g.nx; d.ny = g.ny; d.nz = g.nz;
    d.cell0 = L.NT; d.ncell = g.ncell;
    d.cblk0 = L.nbcnt;
    L.nbcnt += (g.ncell + BCELLS - 1) / BCELLS;
    // collide tiles: at most one per MIN_TILE cells, whatever the launch shape
    L.ntile_max += (int)((g.ncell + MIN_TILE - 1) / MIN_TILE);
    d.v0_off = L.nv0;
    d.red0 = L.nred;
    int nr = 0;
    for (int pl = 0; pl < NPL; ++pl) {
      d.lay_off[pl] = L.nlay;
      d.lay_n[pl] = (int32_t)g.lay[pl].size();
      if (lay) lay->insert(lay->end(), g.lay[pl].begin(), g.lay[pl].end());
      L.nlay += d.lay_n[pl];
      for (int s = 0; s < d.lay_n[pl]; s += RCHUNK) {
        if (red) red->push_back(RedTab{(int32_t)k, pl, s, std::min(RCHUNK, d.lay_n[pl] - s)});
        ++nr;
      }
    }
    if (nr == 0) {  // the 0D models still advance every step
      if (red) red->push_back(RedTab{(int32_t)k, 0, 0, 0});
      nr = 1;
    }
    d.nred = nr;
    L.nred += nr;
    L.NT += g.ncell;
    L.nv0 += (int64_t)g.nx * g.ny;
    if (inst) inst->push_back(d);
  }
  const size_t n = G.size();
  size_t o = 0;
  L.flags = o; o = align256(o + L.NT);
  // neighbour-type words: read by the 16-bit collide only
  L.nbr = o; o = align256(o + (elem_size(prec) == 2 ? (size_t)L.NT * 8 : 0));
  L.inst = o; o = align256(o + n * sizeof(InstDesc));
  L.ctab = o; o = align256(o + (size_t)std::max(L.ntile_max, 1) * sizeof(CTile));
  L.btab = o; o = align256(o + (size_t)std::max(L.ntile_max, 1) * sizeof(CTile));
  L.lay = o; o = align256(o + (size_t)std::max(L.nlay, 1) * 4);
  L.red = o; o = align256(o + (size_t)L.nred * sizeof(RedTab));
  L.red_part = o; o = align256(o + (size_t)L.nred * 16);
  L.bc = o; o = align256(o + NBC * n * sizeof(BcDev));
  L.st = o; o = align256(o + n * sizeof(InstState));
  L.wave = o; o = align256(o + n * (size_t)wave_cap * NREC * 8);
  L.owave = o; o = align256(o + n * (size_t)wave_cap * NOREC * 8);
  L.v0 = o; o = align256(o + (size_t)L.nv0 * r4_size(prec));
  L.err = o; o = align256(o + n * 4);          // one error word per instance
  L.moved = o; o = align256(o + 4);
  L.walls = o; o = align256(o + n * 4);
  L.cwalls = o; o = align256(o + n * 4);
  L.bmark = o; o = align256(o + L.NT);
  L.btmp = o; o = align256(o + L.NT);
  L.bcnt = o; o = align256(o + (size_t)std::max<int64_t>(L.nbcnt, 1) * 4);
  L.gate = o; o = align256(o + 4);
  L.total = o;
}

struct EventPair {
  hipEvent_t a, b;
};

struct Wall {
  bool on = false;
  int64_t np = 0;
  int nband = 0;
  int margin = 2;
  int64_t band_cap = 0;
  std::vector<int32_t> band;
  std::vector<double> X0;      // rest positions, xyz per point (host copy)
  std::vector<double> Xband;   // positions the band was last built around (host copy)
  double* wss = nullptr;       // device, np doubles: wall shear stress read-back
};

// Instances of similar box volume share launch shapes, chosen by the
// autotuner: collide workgroup size and cells per lane, wall tile shape.
struct SizeClass {
  std::vector<int32_t> inst;   // instance ids, ascending (memory order)
  int bs = 256, cpt = 1, tj = 16, tk = 16;
  bool shaped = false;         // shapes set by lbm_set_launch or the autotuner
};

// One launch: the classes that share a shape (or one class while tuning),
// with their slice of the packed tile table or wall list.
struct LaunchGroup {
  int bs = 256, cpt = 1, tj = 16, tk = 16;
  bool nee = false;            // collide tiles holding cells next to a 0D ghost of an
                               // instance with the normal-neighbour extrapolation
  bool bigbox = false;         // wall tiles staged by the large-box kernel
  int cls = -1;                // the class timed by this launch while tuning
  size_t off = 0;              // first tile / wall entry
  int count = 0;               // tiles / walls
  int wall_tiles = 0;          // tiles of the group's largest wall
};

}  // namespace

struct lbm_ctx {
  int n = 0, prec = 1;
  float scale = 1.0f;
  std::vector<Geometry> geo;
  std::vector<InstDesc> inst;
  Layout L;
  hipStream_t stream = nullptr;
  char* work = nullptr;
  void* pop = nullptr;
  Dev dev;
  int64_t step = 0;
  std::string err;
  std::vector<Wall> wall;
  std::vector<int32_t> walls;
  // band rebuilds on the device: the host copies of the bands (lists, sizes,
  // band bits of the flags, positions they were built around) are out of
  // date until refresh_bands reads them back
  bool bands_stale = false;
  int maxlines[3] = {0, 0, 0};   // most lines along x, y, z of a walled instance
  int maxblk = 0;                // most blocks of BCELLS cells of a walled instance
  std::vector<SizeClass> cls;
  std::vector<LaunchGroup> cgroups, wgroups;
  // overlap of the wall exchange with the bulk collide: a side stream, the
  // band-cell tile table (256-cell tiles holding a band cell) and events
  bool overlap = false;
  bool deterministic = false;   // wall tiles launched colour by colour
  int64_t band_check = 32;     // steps between wall-motion tests (0: never)
  hipStream_t side = nullptr;
  hipEvent_t ev_fork = nullptr, ev_wall = nullptr, ev_join = nullptr, ev_red = nullptr;
  int nbtile = 0;
  // per-class kernel events while tuning: (class, kind 0 collide / 1 wall)
  bool tuning = false;
  std::vector<std::pair<std::pair<int, int>, EventPair>> tune_rec;
  // timing
  bool timing = false;
  std::vector<EventPair> pool;
  std::vector<std::pair<int, EventPair>> recorded;
  int64_t t_launch[NTIMED] = {0, 0, 0, 0, 0};
  double t_ms[NTIMED] = {0, 0, 0, 0, 0};
  // graph
  bool use_graph = true;
  hipGraphExec_t gexec = nullptr;
  hipGraph_t graph = nullptr;
};

namespace {

thread_local std::string g_init_err;  // message of the last failed lbm_init / query

lbm_status fail(lbm_ctx* c, lbm_status s, const std::string& m) {
  if (c) c->err = m;
  return s;
}

#define HIPCHK(ctx, call)                                                         \
  do {                                                                           \
    hipError_t e_ = (call);                                                      \
    if (e_ != hipSuccess) return fail(ctx, LBM_E_DEVICE, std::string(#call ": ") + hipGetErrorString(e_)); \
  } while (0)

void drop_graph(lbm_ctx* c) {
  if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
  if (c->graph) (void)hipGraphDestroy(c->graph);
  c->gexec = nullptr;
  c->graph = nullptr;
}

EventPair get_pair(lbm_ctx* c) {
  if (!c->pool.empty()) {
    EventPair p = c->pool.back();
    c->pool.pop_back();
    return p;
  }
  EventPair p;
  (void)hipEventCreate(&p.a);
  (void)hipEventCreate(&p.b);
  return p;
}

// the wall exchange of every launch group on stream s: one launch per group,
// or in the deterministic mode one per tile colour, in colour order
hipError_t enqueue_wall(lbm_ctx* c, int parity, hipStream_t s) {
  const int32_t* cw = (const int32_t*)(c->work + c->L.cwalls);
  for (const LaunchGroup& G : c->wgroups)
    for (int col = c->deterministic ? 0 : -1; col < (c->deterministic ? WALL_COLOURS : 0); ++col) {
      hipError_t e = launch_wall(c->dev, c->prec, parity, G.tj, G.tk, G.bigbox, cw + G.off, G.count, G.wall_tiles,
                                 col, s);
      if (e != hipSuccess) return e;
    }
  return hipSuccess;
}

hipError_t enqueue_step(lbm_ctx* c, int parity, bool timed) {
  hipError_t e;
  EventPair ev[NTIMED];
  auto pre = [&](int k) {
    if (timed) { ev[k] = get_pair(c); (void)hipEventRecord(ev[k].a, c->stream); }
  };
  auto post = [&](int k) {
    if (timed) { (void)hipEventRecord(ev[k].b, c->stream); c->recorded.push_back({k, ev[k]}); }
  };
  auto tpre = [&](EventPair& p) {
    if (c->tuning) { p = get_pair(c); (void)hipEventRecord(p.a, c->stream); }
  };
  auto tpost = [&](EventPair& p, int q, int kind) {
    if (c->tuning) { (void)hipEventRecord(p.b, c->stream); c->tune_rec.push_back({{q, kind}, p}); }
  };
  const CTile* tab = (const CTile*)(c->work + c->L.ctab);
  const int32_t* cw = (const int32_t*)(c->work + c->L.cwalls);
  if (c->dev.nwall > 0 && c->overlap && c->side && !timed && !c->tuning) {
    // main stream: 0D reductions, then the collide of cells outside the
    // wall band; side stream: band moments, wall exchange, membrane.  The
    // band cells collide on the main stream once the wall force is spread.
    hipStream_t s2 = c->side;
    if ((e = hipEventRecord(c->ev_fork, c->stream)) != hipSuccess) return e;
    if ((e = hipStreamWaitEvent(s2, c->ev_fork, 0)) != hipSuccess) return e;
    if ((e = launch_band(c->dev, c->prec, parity, s2)) != hipSuccess) return e;
    if ((e = enqueue_wall(c, parity, s2)) != hipSuccess) return e;
    if ((e = hipEventRecord(c->ev_wall, s2)) != hipSuccess) return e;
    if ((e = launch_membrane(c->dev, parity, s2)) != hipSuccess) return e;
    if ((e = hipEventRecord(c->ev_join, s2)) != hipSuccess) return e;
    if ((e = launch_reduce(c->dev, c->prec, parity, c->L.nred, c->stream)) != hipSuccess) return e;
    for (const LaunchGroup& G : c->cgroups)
      if ((e = launch_collide(c->dev, c->prec, parity, G.bs, G.cpt, G.nee, tab + G.off, G.count, COLLIDE_BULK,
                              c->stream)) != hipSuccess)
        return e;
    if ((e = hipStreamWaitEvent(c->stream, c->ev_wall, 0)) != hipSuccess) return e;
    if ((e = launch_collide(c->dev, c->prec, parity, 256, 1, c->dev.any_nee != 0,
                            (const CTile*)(c->work + c->L.btab), c->nbtile, COLLIDE_BAND, c->stream)) != hipSuccess)
      return e;
    return hipStreamWaitEvent(c->stream, c->ev_join, 0);
  }
  // Untimed, untuned steps with a side stream and a wall run there, from the
  // step's start, the 0D reductions (beside the band moments and the wall
  // exchange: their chain of dependent memory operations stretches under the
  // band's traffic and would otherwise set the length of a shared launch),
  // then, once the force is spread, the wall's time step (k_membrane: reads
  // the wall state and the force, writes the next displacements, which no
  // collide reads) and the few tiles next to a 0D ghost (the normal-neighbour
  // build; in the AA pattern every cell reads and writes only its own slots)
  // beside the bulk collide.  The bulk collide, which overwrites the
  // mid-length layer the reductions read and, without the normal-neighbour
  // build, reads the 0D state they update, waits for the reductions; the main
  // stream joins the side stream before the step ends.  Without a side
  // stream, untimed steps with a wall run the reductions and the band moments
  // as one launch; timed and tuning steps keep everything in sequence.
  const bool fork = !timed && !c->tuning && c->side != nullptr;
  const bool red_side = fork && c->dev.nwall > 0;
  const bool fused = c->dev.nwall > 0 && !timed && !c->tuning && !red_side;
  bool forked = false;
  auto fork_side = [&]() -> hipError_t {
    if (forked) return hipSuccess;
    forked = true;
    hipError_t r = hipEventRecord(c->ev_fork, c->stream);
    return r != hipSuccess ? r : hipStreamWaitEvent(c->side, c->ev_fork, 0);
  };
  if (red_side) {
    if ((e = fork_side()) != hipSuccess) return e;
    if ((e = launch_reduce(c->dev, c->prec, parity, c->L.nred, c->side)) != hipSuccess) return e;
    if ((e = hipEventRecord(c->ev_red, c->side)) != hipSuccess) return e;
  } else if (fused) {
    e = launch_reduce_band(c->dev, c->prec, parity, c->L.nred, c->stream);
    if (e != hipSuccess) return e;
  } else {
    pre(1);
    e = launch_reduce(c->dev, c->prec, parity, c->L.nred, c->stream);
    if (e != hipSuccess) return e;
    post(1);
  }
  if (c->dev.nwall > 0 && !fused) {
    pre(2);
    e = launch_band(c->dev, c->prec, parity, c->stream);
    if (e != hipSuccess) return e;
    post(2);
  }
  if (c->dev.nwall > 0) {
    pre(3);
    for (const LaunchGroup& G : c->wgroups) {
      EventPair p;
      tpre(p);
      for (int col = c->deterministic ? 0 : -1; col < (c->deterministic ? WALL_COLOURS : 0); ++col) {
        e = launch_wall(c->dev, c->prec, parity, G.tj, G.tk, G.bigbox, cw + G.off, G.count, G.wall_tiles, col,
                        c->stream);
        if (e != hipSuccess) return e;
      }
      tpost(p, G.cls, 1);
    }
    if (fork) {
      if ((e = hipEventRecord(c->ev_wall, c->stream)) != hipSuccess) return e;
      if ((e = hipStreamWaitEvent(c->side, c->ev_wall, 0)) != hipSuccess) return e;
      e = launch_membrane(c->dev, parity, c->side);
    } else {
      e = launch_membrane(c->dev, parity, c->stream);
    }
    if (e != hipSuccess) return e;
    post(3);
  }
  pre(0);
  if (fork)
    for (const LaunchGroup& G : c->cgroups) {
      if (!G.nee) continue;
      if ((e = fork_side()) != hipSuccess) return e;
      e = launch_collide(c->dev, c->prec, parity, G.bs, G.cpt, true, tab + G.off, G.count, COLLIDE_ALL, c->side);
      if (e != hipSuccess) return e;
    }
  if (forked && (e = hipEventRecord(c->ev_join, c->side)) != hipSuccess) return e;
  if (red_side && (e = hipStreamWaitEvent(c->stream, c->ev_red, 0)) != hipSuccess) return e;
  // timed steps: the tiles without extrapolation first (id 0), then the
  // others (id 4)
  for (int v = 0; v < 2; ++v) {
    bool any = false;
    for (const LaunchGroup& G : c->cgroups) {
      if ((fork && G.nee) || G.nee != (v == 1)) continue;
      if (!any && v == 1) pre(4);
      any = true;
      EventPair p;
      tpre(p);
      e = launch_collide(c->dev, c->prec, parity, G.bs, G.cpt, G.nee, tab + G.off, G.count, COLLIDE_ALL, c->stream);
      if (e != hipSuccess) return e;
      tpost(p, G.cls, 0);
    }
    if (v == 0) {
      if (forked && (e = hipStreamWaitEvent(c->stream, c->ev_join, 0)) != hipSuccess) return e;
      post(0);
    } else if (any) {
      post(4);
    }
  }
  return hipSuccess;
}

void collect_times(lbm_ctx* c) {
  for (auto& r : c->recorded) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, r.second.a, r.second.b) == hipSuccess) {
      c->t_ms[r.first] += ms;
      c->t_launch[r.first] += 1;
    }
    c->pool.push_back(r.second);
  }
  c->recorded.clear();
}

// Size classes: instances sorted by cell count, split into quartiles (a
// single class below 8 instances).
void make_classes(lbm_ctx* c) {
  const int n = c->n;
  std::vector<int32_t> order(n);
  for (int k = 0; k < n; ++k) order[k] = k;
  std::stable_sort(order.begin(), order.end(),
                   [&](int32_t a, int32_t b) { return c->inst[a].ncell < c->inst[b].ncell; });
  const int nc = n >= 8 ? 4 : 1;
  c->cls.assign(nc, SizeClass());
  for (int q = 0; q < nc; ++q) {
    SizeClass& K = c->cls[q];
    for (int r = q * n / nc; r < (q + 1) * n / nc; ++r) K.inst.push_back(order[r]);
    std::sort(K.inst.begin(), K.inst.end());
  }
}

// Launch groups from the classes' shapes: one collide launch per distinct
// (workgroup, cells per lane) and one wall launch per distinct tile width,
// or one of each per class (per_class, for timing them apart).  Packs and
// uploads the tile table and the wall list.
// Largest stencil box (cells) of wall i's tiles of tj x tk points at the
// positions its band was last built around, and whether that needs the
// large-box wall kernel: some box exceeds 90 % of the standard staging
// capacity (coarse meshes, or a wall whose motion has stretched its tiles;
// the margin leaves room for the motion until the next band build).  One
// tile on the unstaged path (stencils read and spread in global memory) sets
// the whole launch's duration, so a single one is enough to switch.
int64_t wall_max_box(const lbm_ctx* c, int i, int tj, int tk) {
  const InstDesc& d = c->inst[i];
  const std::vector<double>& X = c->wall[i].Xband;
  const int nth = d.nth, nzl = d.nzl;
  int64_t most = 0;
  for (int k0 = 0; k0 < nzl; k0 += tk)
    for (int j0 = 0; j0 < nth; j0 += tj) {
      int lo[3] = {INT32_MAX, INT32_MAX, INT32_MAX}, hi[3] = {INT32_MIN, INT32_MIN, INT32_MIN};
      for (int k = k0; k < std::min(k0 + tk, nzl); ++k)
        for (int j = j0; j < std::min(j0 + tj, nth); ++j)
          for (int a = 0; a < 3; ++a) {
            const int b = (int)std::floor(X[3 * (j + (size_t)nth * k) + a]) - 1;
            lo[a] = std::min(lo[a], b);
            hi[a] = std::max(hi[a], b);
          }
      int64_t vol = 1;
      for (int a = 0; a < 3; ++a) vol *= (int64_t)(hi[a] - lo[a] + 4);
      most = std::max(most, vol);
    }
  return most;
}

bool wall_needs_bigbox(const lbm_ctx* c, int i, int tj, int tk) {
  return wall_max_box(c, i, tj, tk) > wall_boxcap(c->prec == 0 ? 8 : 4, tj) * 9 / 10;
}

lbm_status refresh_bands(lbm_ctx* c);

lbm_status build_groups(lbm_ctx* c, bool per_class) {
  if (lbm_status r = refresh_bands(c)) return r;
  const int nc = (int)c->cls.size();
  std::vector<CTile> tab;
  std::vector<int32_t> walls;
  c->cgroups.clear();
  c->wgroups.clear();
  std::vector<bool> done(nc, false), wdone(nc, false);
  // The tiles that hold a cell next to a 0D ghost of an instance with the
  // normal-neighbour extrapolation go to a launch of their own, the only one
  // built with that variant (it needs more registers, which would cost every
  // other tile occupancy).
  for (int q = 0; q < nc; ++q) {
    if (done[q]) continue;
    LaunchGroup G;
    G.bs = c->cls[q].bs;
    G.cpt = c->cls[q].cpt;
    G.cls = q;
    const int64_t span = (int64_t)G.bs * G.cpt;
    std::vector<CTile> plain, nee;
    for (int r = q; r < nc; ++r) {
      if (done[r] || (r != q && (per_class || c->cls[r].bs != G.bs || c->cls[r].cpt != G.cpt))) continue;
      done[r] = true;
      for (int32_t i : c->cls[r].inst) {
        const std::vector<int32_t>& gn = c->geo[i].ghost_near;
        for (int64_t s = 0; s < c->inst[i].ncell; s += span) {
          auto it = std::lower_bound(gn.begin(), gn.end(), (int32_t)s);
          (it != gn.end() && *it < s + span ? nee : plain).push_back(CTile{i, (int32_t)s});
        }
      }
    }
    for (int v = 0; v < 2; ++v) {
      const std::vector<CTile>& part = v ? nee : plain;
      if (part.empty()) continue;
      LaunchGroup H = G;
      H.nee = v == 1;
      H.off = tab.size();
      tab.insert(tab.end(), part.begin(), part.end());
      H.count = (int)part.size();
      c->cgroups.push_back(H);
    }
  }
  for (int q = 0; q < nc; ++q) {
    if (wdone[q]) continue;
    LaunchGroup G;
    G.tj = c->cls[q].tj;
    G.tk = c->cls[q].tk;
    G.cls = q;
    G.off = walls.size();
    const int tk = G.tk;
    for (int r = q; r < nc; ++r) {
      if (wdone[r] || (r != q && (per_class || c->cls[r].tj != G.tj || c->cls[r].tk != G.tk))) continue;
      wdone[r] = true;
      for (int32_t i : c->cls[r].inst)
        if (c->wall[i].on) {
          walls.push_back(i);
          const InstDesc& d = c->inst[i];
          G.wall_tiles = std::max(G.wall_tiles, ((d.nth + G.tj - 1) / G.tj) * ((d.nzl + tk - 1) / tk));
          G.bigbox = G.bigbox || wall_needs_bigbox(c, i, G.tj, G.tk);
        }
    }
    G.count = (int)(walls.size() - G.off);
    if (G.count > 0) c->wgroups.push_back(G);
  }
  // tiles of 256 cells that hold a band cell, for the band-only collide pass
  std::vector<CTile> btab;
  for (int i = 0; i < c->n; ++i) {
    if (!c->wall[i].on) continue;
    int32_t last = -1;
    for (int32_t cell : c->wall[i].band) {   // ascending
      const int32_t t = cell / 256;
      if (t != last) btab.push_back(CTile{i, t * 256});
      last = t;
    }
  }
  if ((int64_t)btab.size() > c->L.ntile_max) return fail(c, LBM_E_STATE, "band tile table overflow");
  c->nbtile = (int)btab.size();
  if (!btab.empty())
    HIPCHK(c, hipMemcpy(c->work + c->L.btab, btab.data(), btab.size() * sizeof(CTile), hipMemcpyHostToDevice));
  if ((int64_t)tab.size() > c->L.ntile_max) return fail(c, LBM_E_STATE, "tile table overflow");
  if (!tab.empty())
    HIPCHK(c, hipMemcpy(c->work + c->L.ctab, tab.data(), tab.size() * sizeof(CTile), hipMemcpyHostToDevice));
  if (!walls.empty())
    HIPCHK(c, hipMemcpy(c->work + c->L.cwalls, walls.data(), walls.size() * 4, hipMemcpyHostToDevice));
  return LBM_OK;
}

int band_from_points(const Geometry& g, const double* X, int64_t np, int m, bool strict, std::vector<int32_t>& band,
                     std::string& err);

// Read the bands the device rebuilt back into the host copies (band lists,
// sizes, band bits of the flags, positions they were built around).
lbm_status refresh_bands(lbm_ctx* c) {
  if (!c->bands_stale) return LBM_OK;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  std::vector<InstDesc> dd((size_t)c->n);
  HIPCHK(c, hipMemcpy(dd.data(), c->work + c->L.inst, dd.size() * sizeof(InstDesc), hipMemcpyDeviceToHost));
  std::vector<uint8_t> fl((size_t)c->L.NT);
  HIPCHK(c, hipMemcpy(fl.data(), c->work + c->L.flags, fl.size(), hipMemcpyDeviceToHost));
  for (int k = 0; k < c->n; ++k) {
    Wall& W = c->wall[k];
    if (!W.on) continue;
    InstDesc& d = c->inst[k];
    d.nband = dd[k].nband;
    W.nband = d.nband;
    W.band.resize((size_t)d.nband);
    if (d.nband) HIPCHK(c, hipMemcpy(W.band.data(), d.band, (size_t)d.nband * 4, hipMemcpyDeviceToHost));
    std::memcpy(c->geo[k].flags.data(), fl.data() + d.cell0, (size_t)d.ncell);
    std::vector<double> Dr((size_t)d.np * 4);
    HIPCHK(c, hipMemcpy(Dr.data(), d.Dref, (size_t)d.np * 32, hipMemcpyDeviceToHost));
    W.Xband.resize((size_t)d.np * 3);
    for (int64_t p = 0; p < d.np; ++p)
      for (int a = 0; a < 3; ++a) W.Xband[3 * p + a] = W.X0[3 * p + a] + Dr[4 * p + a];
  }
  c->bands_stale = false;
  return LBM_OK;
}

// Rebuild the band of every wall around its current positions X0 + D^n
// (D^n is in Xab[step & 1]) and restart the motion measure from there.
lbm_status rebuild_bands(lbm_ctx* c) {
  if (lbm_status r = refresh_bands(c)) return r;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  std::vector<uint32_t> ierr((size_t)c->n);
  HIPCHK(c, hipMemcpy(ierr.data(), c->work + c->L.err, ierr.size() * 4, hipMemcpyDeviceToHost));
  // In a batch a wall whose band cannot be rebuilt freezes its instance
  // (the error word says why) and the others go on; a single instance
  // reports the failure.
  auto freeze = [&](int k, uint32_t bit, lbm_status code, const std::string& why) -> lbm_status {
    if (c->n == 1) return fail(c, code, why);
    ierr[k] |= bit | ERR_FROZEN;
    HIPCHK(c, hipMemcpy(c->work + c->L.err + (size_t)k * 4, &ierr[k], 4, hipMemcpyHostToDevice));
    return LBM_OK;
  };
  int maxb = 0;
  for (int k = 0; k < c->n; ++k) {
    Wall& W = c->wall[k];
    if (!W.on) continue;
    if (ierr[k]) {   // frozen: its band stays as it was
      maxb = std::max(maxb, W.nband);
      continue;
    }
    InstDesc& d = c->inst[k];
    Geometry& g = c->geo[k];
    const int64_t np = d.np;
    std::vector<double> D4((size_t)np * 4), X((size_t)np * 3);
    double* Dn = d.Xab[c->step & 1];
    HIPCHK(c, hipMemcpy(D4.data(), Dn, (size_t)np * 32, hipMemcpyDeviceToHost));
    for (int64_t p = 0; p < np; ++p)
      for (int q = 0; q < 3; ++q) X[3 * p + q] = W.X0[3 * p + q] + D4[4 * p + q];
    std::vector<int32_t> band;
    std::string why;
    const bool finite = band_from_points(g, X.data(), np, W.margin, false, band, why) == 1;
    if (!finite || (int64_t)band.size() > W.band_cap) {
      const lbm_status fs = !finite ? freeze(k, ERR_NONFINITE, LBM_E_UNSTABLE, "band rebuild: " + why)
                                    : freeze(k, ERR_BAND, LBM_E_BAND, "band rebuild: the band outgrew its capacity");
      if (fs != LBM_OK) return fs;
      maxb = std::max(maxb, W.nband);
      continue;
    }
    for (auto& t : g.flags) t &= (uint8_t)~F_BAND;
    for (int32_t cell : band) g.flags[cell] |= F_BAND;
    HIPCHK(c, hipMemcpy(c->work + c->L.flags + d.cell0, g.flags.data(), g.ncell, hipMemcpyHostToDevice));
    if (!band.empty()) HIPCHK(c, hipMemcpy(d.band, band.data(), band.size() * 4, hipMemcpyHostToDevice));
    HIPCHK(c, hipMemcpy(d.Dref, Dn, (size_t)np * 32, hipMemcpyDeviceToDevice));
    d.nband = (int32_t)band.size();
    HIPCHK(c, hipMemcpy(c->work + c->L.inst + k * sizeof(InstDesc), &d, sizeof d, hipMemcpyHostToDevice));
    W.band.swap(band);
    W.nband = d.nband;
    W.Xband.swap(X);
    maxb = std::max(maxb, W.nband);
  }
  HIPCHK(c, hipMemset(c->work + c->L.moved, 0, 4));
  (void)maxb;
  drop_graph(c);
  return build_groups(c, false);
}

// Wall-motion test: once a point has moved m - 1 lattice units (m = band
// margin) since its band was built, the band is rebuilt, so that no stencil
// reaches past it as long as no point moves a whole unit between tests.
// The test and the rebuild run on the device without a host round trip (a
// gate word decides); with the overlap of the wall exchange on (its
// band-only collide pass needs the host's band lists) the host waits for the
// motion word and rebuilds on the host.
lbm_status check_bands(lbm_ctx* c) {
  int m = 1 << 30;
  for (int k = 0; k < c->n; ++k)
    if (c->wall[k].on) m = std::min(m, c->wall[k].margin);
  if (m == (1 << 30)) return LBM_OK;
  if (!c->overlap) {
    HIPCHK(c, launch_motion(c->dev, (int)(c->step & 1), c->stream));
    HIPCHK(c, launch_band_rebuild(c->dev, (int)(c->step & 1), (float)(m - 1), c->maxlines, c->maxblk, c->stream));
    c->bands_stale = true;
    return LBM_OK;
  }
  HIPCHK(c, launch_motion(c->dev, (int)(c->step & 1), c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  uint32_t bits = 0;
  HIPCHK(c, hipMemcpy(&bits, c->work + c->L.moved, 4, hipMemcpyDeviceToHost));
  float moved;
  std::memcpy(&moved, &bits, 4);
  if (!(moved < (float)(m - 1))) return rebuild_bands(c);
  return LBM_OK;
}

template <class T>
lbm_status h2d(lbm_ctx* c, size_t off, const T* src, size_t count) {
  if (count == 0) return LBM_OK;
  HIPCHK(c, hipMemcpyAsync(c->work + off, src, count * sizeof(T), hipMemcpyHostToDevice, c->stream));
  return LBM_OK;
}

// Read the raw storage of instance k into host doubles, AoS [cell][19],
// undoing the AA parity permutation.
// Steps instance k has taken: the context's count, or, for an instance that
// failed and was frozen, the count it stopped at (its state is at that step).
lbm_status inst_step(lbm_ctx* c, int k, int64_t* t) {
  HIPCHK(c, hipStreamSynchronize(c->stream));
  InstState st;
  HIPCHK(c, hipMemcpy(&st, c->work + c->L.st + (size_t)k * sizeof(InstState), sizeof st, hipMemcpyDeviceToHost));
  *t = st.step;
  return LBM_OK;
}

lbm_status inst_live(lbm_ctx* c, int k) {
  HIPCHK(c, hipStreamSynchronize(c->stream));
  uint32_t e = 0;
  HIPCHK(c, hipMemcpy(&e, c->work + c->L.err + (size_t)k * 4, 4, hipMemcpyDeviceToHost));
  if (e) return fail(c, LBM_E_STATE, "instance " + std::to_string(k) + " has failed and is frozen");
  return LBM_OK;
}

lbm_status read_pops(lbm_ctx* c, int k, std::vector<double>& out) {
  const Geometry& g = c->geo[k];
  const InstDesc& d = c->inst[k];
  const int es = elem_size(c->prec);
  std::vector<char> raw((size_t)NQ * g.ncell * es);
  HIPCHK(c, hipStreamSynchronize(c->stream));
  for (int i = 0; i < NQ; ++i)
    HIPCHK(c, hipMemcpy(raw.data() + (size_t)i * g.ncell * es,
                        (char*)c->pop + ((size_t)i * c->L.NT + d.cell0) * es, (size_t)g.ncell * es,
                        hipMemcpyDeviceToHost));
  auto val = [&](int i, int64_t cell) -> double {
    const char* p = raw.data() + ((size_t)i * g.ncell + cell) * es;
    switch (c->prec) {
      case 0: { double v; std::memcpy(&v, p, 8); return v; }
      case 1: { float v; std::memcpy(&v, p, 4); return v; }
      case 2: { uint16_t u; std::memcpy(&u, p, 2); return (double)(f16_to_f32(u) * (1.0f / c->scale)); }
      default: { uint16_t u; std::memcpy(&u, p, 2); return (double)(bf16_to_f32(u) * (1.0f / c->scale)); }
    }
  };
  const int64_t sy = g.nx, sz = (int64_t)g.nx * g.ny;
  int64_t tk = 0;
  lbm_status r = inst_step(c, k, &tk);
  if (r != LBM_OK) return r;
  const bool odd = tk & 1;
  out.assign((size_t)g.ncell * NQ, 0.0);
  for (int64_t cell = 0; cell < g.ncell; ++cell) {
    if ((g.flags[cell] & TYPE_MASK) != T_FLUID) continue;
    for (int i = 0; i < NQ; ++i) {
      double v;
      if (!odd) {
        v = val(i, cell);
      } else {
        // streamed, bounced-back or extrapolated: all at A[opp i][c - e_i]
        v = val(OPPh[i], cell - (EXh[i] + EYh[i] * sy + EZh[i] * sz));
      }
      out[(size_t)cell * NQ + i] = v + W[i] * d.dref;
    }
  }
  return LBM_OK;
}

// Band of a wall (fluid cells within margin m of the 4x4x4 stencils of the
// points X, xyz per point): the stencil base cells b = floor(X) - 1 are
// marked, then the marks are dilated by [b - m, b + 3 + m] along x, y and z
// in turn (one running window per line).
// strict: every stencil must lie inside the box (registration); otherwise a
// base outside the box is clamped to it (a rebuilt band; stencil cells
// outside the box take no part in the exchange).  Returns 1 on success, 0
// for a stencil outside the box (strict) and -1 for a non-finite point.
int band_from_points(const Geometry& g, const double* X, int64_t np, int m, bool strict, std::vector<int32_t>& band,
                     std::string& err) {
  std::vector<uint8_t> a(g.ncell, 0), t(g.ncell, 0);
  const int n3[3] = {g.nx, g.ny, g.nz};
  for (int64_t p = 0; p < np; ++p) {
    int b[3];
    for (int q = 0; q < 3; ++q) {
      const double v = X[3 * p + q];
      if (!std::isfinite(v) || std::fabs(v) > 1e9) { err = "non-finite wall point"; return -1; }
      b[q] = (int)std::floor(v) - 1;
      if (b[q] < 0 || b[q] + 3 > n3[q] - 1) {
        if (strict) { err = "wall stencil touches the box faces"; return 0; }
        b[q] = std::min(std::max(b[q], 0), n3[q] - 1);
      }
    }
    a[b[0] + (int64_t)g.nx * (b[1] + (int64_t)g.ny * b[2])] = 1;
  }
  const int64_t stride[3] = {1, g.nx, (int64_t)g.nx * g.ny};
  for (int ax = 0; ax < 3; ++ax) {
    const int n = n3[ax];
    const int64_t s = stride[ax];
    // lines along ax: every cell whose ax-coordinate is 0 starts one
    for (int64_t c0 = 0; c0 < g.ncell; ++c0) {
      if ((c0 / s) % n != 0) continue;
      // cell i is covered by a base in [i - 3 - m, i + m]
      int cnt = 0;
      for (int i = -3 - m; i < n; ++i) {
        const int add = i + m, drop = i - 4 - m;   // window [i - 3 - m, i + m]
        if (add >= 0 && add < n) cnt += a[c0 + add * s];
        if (drop >= 0 && drop < n) cnt -= a[c0 + drop * s];
        if (i >= 0) t[c0 + i * s] = cnt > 0;
      }
    }
    a.swap(t);
  }
  band.clear();
  for (int64_t cell = 0; cell < g.ncell; ++cell)
    if (a[cell] && (g.flags[cell] & TYPE_MASK) == T_FLUID) band.push_back((int32_t)cell);
  return 1;
}

bool wall_band(const lbm_ctx* c, int k, const lbm_wall_desc* w, std::vector<int32_t>& band, std::string& err) {
  const int m = w->band_margin > 0 ? w->band_margin : 2;
  return band_from_points(c->geo[k], w->X0_host, (int64_t)w->n_theta * w->n_z, m, true, band, err) == 1;
}

// band list capacity reserved in the wall buffer (the band grows when the
// wall dilates and the band is rebuilt)
int64_t band_capacity(int64_t nband) { return 2 * nband + 4096; }

struct FsiLayout {
  size_t u4, b4, X0, Xa, Xb, slip, Vf, Fp, band, Dref, wss, total;
};
FsiLayout fsi_plan(int64_t ncell, int64_t np, int64_t nband, int prec) {
  FsiLayout f;
  const size_t r4 = r4_size(prec);
  size_t o = 0;
  f.u4 = o; o = align256(o + ncell * r4);
  f.b4 = o; o = align256(o + ncell * r4);
  f.X0 = o; o = align256(o + np * 32);
  f.Xa = o; o = align256(o + np * 32);
  f.Xb = o; o = align256(o + np * 32);
  f.slip = o; o = align256(o + np * 32);
  f.Vf = o; o = align256(o + np * r4);
  f.Fp = o; o = align256(o + np * 32);
  f.band = o; o = align256(o + band_capacity(nband) * 4);
  f.Dref = o; o = align256(o + np * 32);
  f.wss = o; o = align256(o + np * 8);        // wall shear stress read-back
  f.total = o;
  return f;
}

bool valid_wall(const lbm_wall_desc* w, std::string& err) {
  if (!w || !w->X0_host) { err = "wall descriptor or X0 is NULL"; return false; }
  if (w->n_theta < 3 || w->n_z < 2) { err = "wall mesh needs n_theta >= 3 and n_z >= 2"; return false; }
  if (!(w->ds_theta > 0 && w->ds_z > 0 && w->area > 0 && w->mass > 0)) {
    err = "wall spacings, area and mass must be positive";
    return false;
  }
  if (w->kernel < 0 || w->kernel > 1 || w->mode < 0 || w->mode > 1 || w->shell < 0 || w->shell > 1) {
    err = "wall kernel, mode and shell must be 0 or 1";
    return false;
  }
  if (w->shell == 1 && !(w->poisson > -1.0 && w->poisson < 1e6)) {
    err = "the shell model needs a Poisson ratio above -1";
    return false;
  }
  return true;
}

}  // namespace

// ===========================================================================
extern "C" {

lbm_status lbm_query_sizes(const lbm_config* cfgs, int32_t n, size_t* pop_bytes, size_t* work_bytes) {
  if (!cfgs || n <= 0 || !pop_bytes || !work_bytes) return LBM_E_INVAL;
  std::vector<Geometry> G(n);
  for (int k = 0; k < n; ++k)
    if (!build_geometry(cfgs[k], G[k], g_init_err)) return LBM_E_INVAL;
  const int prec = cfgs[0].precision;
  if (prec < 0 || prec > 3) return LBM_E_INVAL;
  Layout L;
  plan(G, prec, cfgs[0].wave_cap > 0 ? cfgs[0].wave_cap : 4096, L, nullptr, nullptr, nullptr);
  if (L.NT >= ((int64_t)1 << 31)) {  // the kernels index cells with 32 bits
    g_init_err = "more than 2^31 - 1 cells in one context";
    return LBM_E_INVAL;
  }
  if (L.NT * elem_size(prec) >= ((int64_t)1 << 32)) {  // 32-bit byte offsets per direction
    g_init_err = "one direction's populations exceed 4 GiB";
    return LBM_E_INVAL;
  }
  *pop_bytes = (size_t)NQ * L.NT * elem_size(prec);
  *work_bytes = L.total;
  return LBM_OK;
}

lbm_status lbm_init(const lbm_config* cfgs, int32_t n, const lbm_buffers* buf, void* hip_stream, lbm_ctx** out) {
  if (!out) return LBM_E_INVAL;
  *out = nullptr;
  if (!cfgs || n <= 0 || !buf || !buf->pop || !buf->work) return LBM_E_INVAL;
  lbm_ctx* c = new lbm_ctx();
  c->n = n;
  c->prec = cfgs[0].precision;
  if (c->prec < 0 || c->prec > 3) { delete c; return LBM_E_INVAL; }
  for (int k = 1; k < n; ++k)
    if (cfgs[k].precision != c->prec) { delete c; return LBM_E_INVAL; }
  c->geo.resize(n);
  for (int k = 0; k < n; ++k)
    if (!build_geometry(cfgs[k], c->geo[k], g_init_err)) { delete c; return LBM_E_INVAL; }
  double s = cfgs[0].store_scale;
  if (c->prec == 2 && s == 0.0) s = 256.0;
  if (c->prec <= 1 || s == 0.0) s = 1.0;
  int ex;
  if (std::frexp(s, &ex) != 0.5) { delete c; return LBM_E_INVAL; }  // power of two only
  c->scale = (float)s;
  std::vector<int32_t> lay;
  std::vector<RedTab> red;
  plan(c->geo, c->prec, cfgs[0].wave_cap > 0 ? cfgs[0].wave_cap : 4096, c->L, &c->inst, &lay, &red);
  if (c->L.NT >= ((int64_t)1 << 31)) {  // the kernels index cells with 32 bits
    g_init_err = "more than 2^31 - 1 cells in one context";
    delete c;
    return LBM_E_INVAL;
  }
  if (c->L.NT * elem_size(c->prec) >= ((int64_t)1 << 32)) {  // 32-bit byte offsets per direction
    g_init_err = "one direction's populations exceed 4 GiB";
    delete c;
    return LBM_E_INVAL;
  }
  for (int k = 0; k < n; ++k) {
    c->inst[k].tau = cfgs[k].tau;
    c->inst[k].omega = 1.0 / cfgs[k].tau;
    c->inst[k].nee = cfgs[k].nee_variant;
    c->inst[k].dref = 3.0 * cfgs[k].p_ref;
  }
  if (buf->pop_bytes < (size_t)NQ * c->L.NT * elem_size(c->prec) || buf->work_bytes < c->L.total) {
    delete c;
    return LBM_E_INVAL;
  }
  c->stream = (hipStream_t)hip_stream;
  c->work = (char*)buf->work;
  c->pop = buf->pop;
  c->wall.resize(n);

  Dev& d = c->dev;
  std::memset(&d, 0, sizeof d);
  d.pop = c->pop;
  d.NT = c->L.NT;
  d.scale = c->scale;
  d.inv_scale = 1.0f / c->scale;
  d.flags = (const uint8_t*)(c->work + c->L.flags);
  d.nbr = (const uint64_t*)(c->work + c->L.nbr);
  d.inst = (const InstDesc*)(c->work + c->L.inst);
  d.lay = (const int32_t*)(c->work + c->L.lay);
  d.red = (const RedTab*)(c->work + c->L.red);
  d.red_part = (double*)(c->work + c->L.red_part);
  d.bc = (BcDev*)(c->work + c->L.bc);
  d.st = (InstState*)(c->work + c->L.st);
  d.wave = (double*)(c->work + c->L.wave);
  d.wave_cap = c->L.wave_cap;
  d.v0 = c->work + c->L.v0;
  d.err = (uint32_t*)(c->work + c->L.err);
  d.owave = (double*)(c->work + c->L.owave);
  d.moved = (uint32_t*)(c->work + c->L.moved);
  d.slotcnt = nullptr;
  d.bmark = (uint8_t*)(c->work + c->L.bmark);
  d.btmp = (uint8_t*)(c->work + c->L.btmp);
  d.bcnt = (int32_t*)(c->work + c->L.bcnt);
  d.gate = (uint32_t*)(c->work + c->L.gate);
  d.walls = (const int32_t*)(c->work + c->L.walls);
  d.nwall = 0;
  for (int k = 0; k < n; ++k) d.any_nee |= cfgs[k].nee_variant;

  std::vector<uint8_t> flags(c->L.NT);
  for (int k = 0; k < n; ++k)
    std::memcpy(flags.data() + c->inst[k].cell0, c->geo[k].flags.data(), c->geo[k].ncell);
  std::vector<BcDev> bc(NBC * n);
  for (int k = 0; k < NBC * n; ++k) {
    std::memset(&bc[k], 0, sizeof(BcDev));
    bc[k].kind = BC_PRESSURE;
    bc[k].boundary = k % NBC;
    bc[k].Td = -1;
  }
  std::vector<InstState> st(n);
  std::memset(st.data(), 0, n * sizeof(InstState));
  // Tables go up with synchronous copies (init is not on the hot path, and
  // the host vectors die with this call); then clear and fill on the stream.
  auto up = [&](size_t off, const void* src, size_t bytes) -> hipError_t {
    return bytes ? hipMemcpy(c->work + off, src, bytes, hipMemcpyHostToDevice) : hipSuccess;
  };
  hipError_t e = hipStreamSynchronize(c->stream);
  const char* what = "hipStreamSynchronize";
  if (e == hipSuccess) { e = up(c->L.flags, flags.data(), flags.size()); what = "flags upload"; }
  for (int k = 0; k < n && e == hipSuccess; ++k) {
    if (elem_size(c->prec) == 2) {
      e = up(c->L.nbr + (size_t)c->inst[k].cell0 * 8, c->geo[k].nbr.data(), (size_t)c->geo[k].ncell * 8);
      what = "neighbour-type upload";
    }
    std::vector<uint64_t>().swap(c->geo[k].nbr);   // the device copy (if any) from here on
  }
  if (e == hipSuccess) { e = up(c->L.inst, c->inst.data(), c->inst.size() * sizeof(InstDesc)); what = "instance upload"; }
  if (e == hipSuccess) { e = up(c->L.lay, lay.data(), lay.size() * 4); what = "layer upload"; }
  if (e == hipSuccess) { e = up(c->L.red, red.data(), red.size() * sizeof(RedTab)); what = "reduction table upload"; }
  if (e == hipSuccess) { e = up(c->L.bc, bc.data(), bc.size() * sizeof(BcDev)); what = "0D state upload"; }
  if (e == hipSuccess) { e = up(c->L.st, st.data(), st.size() * sizeof(InstState)); what = "step state upload"; }
  if (e == hipSuccess) { e = hipMemset(c->work + c->L.err, 0, (size_t)n * 4); what = "error flag clear"; }
  if (e == hipSuccess) { e = hipMemset(c->work + c->L.moved, 0, 4); what = "wall motion clear"; }
  if (e == hipSuccess) {   // the device band rebuild keeps its marks zero between rebuilds
    e = hipMemset(c->work + c->L.bmark, 0, (size_t)(c->L.btmp - c->L.bmark) + (size_t)c->L.NT);
    what = "band marks clear";
  }
  if (e == hipSuccess) { e = hipMemset(c->work + c->L.v0, 0, (size_t)c->L.nv0 * r4_size(c->prec)); what = "snapshot clear"; }
  if (e == hipSuccess) { e = hipMemset(c->work + c->L.wave, 0, (size_t)n * c->L.wave_cap * NREC * 8); what = "waveform clear"; }
  if (e == hipSuccess) {
    e = hipMemset(c->work + c->L.owave, 0, (size_t)n * c->L.wave_cap * NOREC * 8);
    what = "outlet waveform clear";
  }
  for (int k = 0; k < n && e == hipSuccess; ++k) {
    e = launch_fill_rest(d, c->prec, c->inst[k].cell0, c->inst[k].ncell, -c->inst[k].dref, c->stream);
    what = "rest-state fill launch";
  }
  if (e != hipSuccess) {
    g_init_err = std::string(what) + ": " + hipGetErrorString(e);
    (void)hipStreamSynchronize(c->stream);
    delete c;
    return LBM_E_DEVICE;
  }
  make_classes(c);
  if (hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&c->ev_wall, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&c->ev_red, hipEventDisableTiming) != hipSuccess) {
    g_init_err = "side stream or event creation failed";
    (void)hipStreamSynchronize(c->stream);
    delete c;
    return LBM_E_DEVICE;
  }
  if (build_groups(c, false) != LBM_OK) {
    g_init_err = c->err;
    (void)hipStreamSynchronize(c->stream);
    delete c;
    return LBM_E_DEVICE;
  }
  *out = c;
  return LBM_OK;
}

static lbm_status run_steps(lbm_ctx* c, int64_t nsteps);

lbm_status lbm_step(lbm_ctx* c, int64_t nsteps) {
  if (!c) return LBM_E_INVAL;
  if (nsteps < 0) return fail(c, LBM_E_INVAL, "nsteps < 0");
  if (c->dev.nwall == 0 || c->band_check <= 0) return run_steps(c, nsteps);
  // with walls: run up to each multiple of band_check, then test the motion
  int64_t left = nsteps;
  while (left > 0) {
    const int64_t to_check = c->band_check - (c->step % c->band_check);
    const int64_t k = std::min(left, to_check);
    lbm_status s = run_steps(c, k);
    if (s != LBM_OK) return s;
    left -= k;
    if (c->step % c->band_check == 0) {
      s = check_bands(c);
      if (s != LBM_OK) return s;
    }
  }
  return LBM_OK;
}

static lbm_status run_steps(lbm_ctx* c, int64_t nsteps) {
  int64_t left = nsteps;
  const bool graph = c->use_graph && !c->timing && !c->tuning;
  if (graph && left >= 2) {
    if ((c->step & 1) && left > 0) {
      HIPCHK(c, enqueue_step(c, 1, false));
      c->step++;
      left--;
    }
    if (!c->gexec && left >= 2) {
      HIPCHK(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
      hipError_t e0 = enqueue_step(c, 0, false);
      hipError_t e1 = enqueue_step(c, 1, false);
      hipGraph_t gr = nullptr;
      hipError_t e2 = hipStreamEndCapture(c->stream, &gr);
      if (e0 != hipSuccess || e1 != hipSuccess || e2 != hipSuccess)
        return fail(c, LBM_E_DEVICE, "graph capture failed");
      c->graph = gr;
      HIPCHK(c, hipGraphInstantiate(&c->gexec, c->graph, nullptr, nullptr, 0));
    }
    while (left >= 2) {
      HIPCHK(c, hipGraphLaunch(c->gexec, c->stream));
      c->step += 2;
      left -= 2;
    }
  }
  while (left > 0) {
    HIPCHK(c, enqueue_step(c, (int)(c->step & 1), c->timing));
    c->step++;
    left--;
  }
  return LBM_OK;
}

int32_t lbm_num_classes(lbm_ctx* c) { return c ? (int32_t)c->cls.size() : -1; }

lbm_status lbm_class_info(lbm_ctx* c, int32_t q, int32_t* instances, int64_t* cells, int64_t* wall_points) {
  if (!c || q < 0 || q >= (int)c->cls.size()) return LBM_E_INVAL;
  const SizeClass& K = c->cls[q];
  int64_t nc = 0, np = 0;
  for (int32_t i : K.inst) {
    nc += c->inst[i].ncell;
    if (c->wall[i].on) np += c->wall[i].np;
  }
  if (instances) *instances = (int32_t)K.inst.size();
  if (cells) *cells = nc;
  if (wall_points) *wall_points = np;
  return LBM_OK;
}

lbm_status lbm_get_launch(lbm_ctx* c, int32_t q, lbm_launch* out) {
  if (!c || !out || q < 0 || q >= (int)c->cls.size()) return LBM_E_INVAL;
  out->block = c->cls[q].bs;
  out->cells_per_lane = c->cls[q].cpt;
  out->wall_tile_theta = c->cls[q].tj;
  out->wall_tile_z = c->cls[q].tk;
  return LBM_OK;
}

namespace {
// the wall tile shapes (theta x z mesh points) the kernel is built for
constexpr int WALL_TILES[6][2] = {{8, 32}, {16, 16}, {32, 8}, {8, 16}, {16, 8}, {8, 8}};

int tile_z(const lbm_launch* l) { return l->wall_tile_z ? l->wall_tile_z : (l->wall_tile_theta ? 256 / l->wall_tile_theta : 0); }

bool valid_launch(const lbm_launch* l) {
  if (!l || !(l->block == 128 || l->block == 256 || l->block == 512) ||
      !(l->cells_per_lane == 1 || l->cells_per_lane == 2))
    return false;
  for (const auto& t : WALL_TILES)
    if (l->wall_tile_theta == t[0] && tile_z(l) == t[1]) return true;
  return false;
}

void apply_launch(lbm_ctx* c, int q, const lbm_launch& l) {
  SizeClass& K = c->cls[q];
  K.bs = l.block;
  K.cpt = l.cells_per_lane;
  K.tj = l.wall_tile_theta;
  K.tk = tile_z(&l);
  K.shaped = true;
}
}  // namespace

lbm_status lbm_set_launch(lbm_ctx* c, int32_t q, const lbm_launch* l) {
  if (!c || q < 0 || q >= (int)c->cls.size()) return LBM_E_INVAL;
  if (!valid_launch(l)) return fail(c, LBM_E_INVAL,
                "block 128/256/512, 1-2 cells per lane, wall tile 8x32, 16x16, 32x8, 8x16, 16x8 or 8x8");
  HIPCHK(c, hipStreamSynchronize(c->stream));
  drop_graph(c);
  apply_launch(c, q, *l);
  return build_groups(c, false);
}

lbm_status lbm_autotune(lbm_ctx* c, int32_t trial_steps, int64_t* advanced) {
  if (!c) return LBM_E_INVAL;
  if (trial_steps < 2) return fail(c, LBM_E_INVAL, "trial_steps < 2");
  trial_steps += trial_steps & 1;   // whole even/odd pairs
  HIPCHK(c, hipStreamSynchronize(c->stream));
  drop_graph(c);
  const int nc = (int)c->cls.size();
  std::vector<lbm_launch> best(nc);
  for (int q = 0; q < nc; ++q) lbm_get_launch(c, q, &best[q]);
  int64_t ran = 0;
  // time every candidate over trial_steps ordinary steps (after two
  // untimed ones), per class and kernel; phase 0 tunes the collide shape,
  // phase 1 the wall tile with the chosen collide shape
  // cand == nullptr: every class on its own current shape
  auto trial = [&](const lbm_launch* cand, int kind, std::vector<double>& ms) -> lbm_status {
    for (int q = 0; q < nc; ++q) {
      lbm_launch l = best[q];
      if (cand && kind == 0) { l.block = cand->block; l.cells_per_lane = cand->cells_per_lane; }
      if (cand && kind == 1) {
        l.wall_tile_theta = cand->wall_tile_theta;
        l.wall_tile_z = cand->wall_tile_z;
      }
      apply_launch(c, q, l);
    }
    lbm_status s = build_groups(c, true);   // one launch per class, timed apart
    if (s != LBM_OK) return s;
    for (int k = 0; k < 2; ++k) {
      HIPCHK(c, enqueue_step(c, (int)(c->step & 1), false));
      c->step++;
    }
    c->tuning = true;
    hipError_t e = hipSuccess;
    for (int k = 0; k < trial_steps && e == hipSuccess; ++k) {
      e = enqueue_step(c, (int)(c->step & 1), false);
      c->step++;
    }
    c->tuning = false;
    ran += 2 + trial_steps;
    HIPCHK(c, e);
    HIPCHK(c, hipStreamSynchronize(c->stream));
    ms.assign(nc, 0.0);
    for (auto& r : c->tune_rec) {
      float t = 0.f;
      if (r.first.second == kind && hipEventElapsedTime(&t, r.second.a, r.second.b) == hipSuccess)
        ms[r.first.first] += t;
      c->pool.push_back(r.second);
    }
    c->tune_rec.clear();
    return LBM_OK;
  };
  // A class keeps its current shape unless a candidate is at least 2 %
  // faster (run-to-run timing noise is about 1 %): the current shapes are
  // timed first in each phase.
  const double gain = 0.98;
  std::vector<double> bms, ms;
  std::vector<lbm_launch> pick = best;
  lbm_status st = trial(nullptr, 0, bms);
  if (st != LBM_OK) return st;
  const int shapes[6][2] = {{128, 1}, {128, 2}, {256, 1}, {256, 2}, {512, 1}, {512, 2}};
  for (auto& sh : shapes) {
    lbm_launch cand = best[0];
    cand.block = sh[0];
    cand.cells_per_lane = sh[1];
    st = trial(&cand, 0, ms);
    if (st != LBM_OK) return st;
    for (int q = 0; q < nc; ++q)
      if (ms[q] < bms[q] * gain) { bms[q] = ms[q]; pick[q].block = sh[0]; pick[q].cells_per_lane = sh[1]; }
  }
  for (int q = 0; q < nc; ++q) { best[q].block = pick[q].block; best[q].cells_per_lane = pick[q].cells_per_lane; }
  if (c->dev.nwall > 0) {
    std::vector<bool> has_wall(nc, false);
    for (int q = 0; q < nc; ++q)
      for (int32_t i : c->cls[q].inst) has_wall[q] = has_wall[q] || c->wall[i].on;
    st = trial(nullptr, 1, bms);
    if (st != LBM_OK) return st;
    for (const auto& t : WALL_TILES) {
      lbm_launch cand = best[0];
      cand.wall_tile_theta = t[0];
      cand.wall_tile_z = t[1];
      st = trial(&cand, 1, ms);
      if (st != LBM_OK) return st;
      for (int q = 0; q < nc; ++q)
        if (has_wall[q] && ms[q] < bms[q] * gain) {
          bms[q] = ms[q];
          pick[q].wall_tile_theta = t[0];
          pick[q].wall_tile_z = t[1];
        }
    }
    for (int q = 0; q < nc; ++q) {
      best[q].wall_tile_theta = pick[q].wall_tile_theta;
      best[q].wall_tile_z = pick[q].wall_tile_z;
    }
  }
  for (int q = 0; q < nc; ++q) apply_launch(c, q, best[q]);
  lbm_status s = build_groups(c, false);
  if (s != LBM_OK) return s;
  if (advanced) *advanced = ran;
  return LBM_OK;
}

lbm_status lbm_couple_0d(lbm_ctx* c, int32_t inst, int32_t b, int32_t kind, const double* params, int32_t np,
                         const double* state, int32_t nst) {
  if (!c) return LBM_E_INVAL;
  if (inst < 0 || inst >= c->n || b < 0 || b >= NBC) return fail(c, LBM_E_INVAL, "bad instance or boundary");
  if (!params && np > 0) return fail(c, LBM_E_INVAL, "params NULL");
  int need = kind == BC_PRESSURE || kind == BC_VELOCITY ? 1 : (kind == BC_WK3 ? 3 : (kind == BC_LV ? 11 : -1));
  if (need < 0) return fail(c, LBM_E_INVAL, "unknown 0D kind");
  if (np < need || np > 16) return fail(c, LBM_E_INVAL, "wrong number of 0D parameters");
  if (kind == BC_LV && b != 0) return fail(c, LBM_E_INVAL, "the LV model couples to the inlet only");
  if (kind == BC_WK3 && b == 2) return fail(c, LBM_E_INVAL, "the exterior takes constant models only");
  if (kind == BC_WK3 && !(params[0] > 0 && params[1] > 0 && params[2] > 0))
    return fail(c, LBM_E_INVAL, "Windkessel Rp, C, Rd must be positive");
  if (kind == BC_LV && !(params[1] > 0 && params[2] > 0 && params[3] > 0 && params[5] > 0))
    return fail(c, LBM_E_INVAL, "LV Emin, Tc, Tmax, N_S must be positive");
  BcDev B;
  std::memset(&B, 0, sizeof B);
  B.kind = kind;
  B.boundary = b;
  for (int k = 0; k < np; ++k) B.par[k] = params[k];
  B.Td = -1;
  if (kind == BC_WK3) B.Pw = (state && nst > 0) ? state[0] : 0.0;
  if (kind == BC_LV) B.Pv = (state && nst > 0) ? state[0] : params[4];
  HIPCHK(c, hipStreamSynchronize(c->stream));
  HIPCHK(c, hipMemcpy(c->work + c->L.bc + (NBC * (size_t)inst + b) * sizeof(BcDev), &B, sizeof B,
                      hipMemcpyHostToDevice));
  return LBM_OK;
}

lbm_status lbm_get_0d(lbm_ctx* c, int32_t inst, int32_t b, double* out) {
  if (!c || !out || inst < 0 || inst >= c->n || b < 0 || b >= NBC) return LBM_E_INVAL;
  BcDev B;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  HIPCHK(c, hipMemcpy(&B, c->work + c->L.bc + (NBC * (size_t)inst + b) * sizeof(BcDev), sizeof B,
                      hipMemcpyDeviceToHost));
  out[0] = B.vmode; out[1] = B.pstar; out[2] = B.S; out[3] = B.Pv;
  out[4] = B.Pw; out[5] = B.open; out[6] = (double)B.Td; out[7] = B.vz;
  return LBM_OK;
}

lbm_status lbm_fsi_query_sizes(lbm_ctx* c, int32_t k, const lbm_wall_desc* w, size_t* bytes) {
  if (!c || !bytes || k < 0 || k >= c->n) return LBM_E_INVAL;
  if (!valid_wall(w, c->err)) return LBM_E_INVAL;
  std::vector<int32_t> band;
  if (!wall_band(c, k, w, band, c->err)) return LBM_E_INVAL;
  *bytes = fsi_plan(c->geo[k].ncell, (int64_t)w->n_theta * w->n_z, (int64_t)band.size(), c->prec).total;
  return LBM_OK;
}

lbm_status lbm_fsi_exchange(lbm_ctx* c, int32_t k, const lbm_wall_desc* w, void* fsi, size_t fsi_bytes) {
  if (!c || k < 0 || k >= c->n || !fsi) return LBM_E_INVAL;
  if (!valid_wall(w, c->err)) return LBM_E_INVAL;
  if (lbm_status r = refresh_bands(c)) return r;
  std::vector<int32_t> band;
  if (!wall_band(c, k, w, band, c->err)) return LBM_E_INVAL;
  Geometry& g = c->geo[k];
  const int64_t np = (int64_t)w->n_theta * w->n_z;
  const FsiLayout f = fsi_plan(g.ncell, np, (int64_t)band.size(), c->prec);
  if (fsi_bytes < f.total) return fail(c, LBM_E_INVAL, "wall buffer too small");
  HIPCHK(c, hipStreamSynchronize(c->stream));
  drop_graph(c);
  // band bits
  for (auto& t : g.flags) t &= (uint8_t)~F_BAND;
  for (int32_t cell : band) g.flags[cell] |= F_BAND;
  char* F = (char*)fsi;
  InstDesc& d = c->inst[k];
  d.has_wall = 1;
  d.nth = w->n_theta;
  d.nzl = w->n_z;
  d.np = np;
  d.nband = (int32_t)band.size();
  d.u4 = F + f.u4;
  d.b4 = F + f.b4;
  d.X0 = (double*)(F + f.X0);
  d.Xab[0] = (double*)(F + f.Xa);
  d.Xab[1] = (double*)(F + f.Xb);
  d.slip = (double*)(F + f.slip);
  d.Vf = F + f.Vf;
  d.Fp = F + f.Fp;
  d.band = (int32_t*)(F + f.band);
  d.Dref = (double*)(F + f.Dref);
  d.ds_th = w->ds_theta; d.ds_z = w->ds_z; d.area = w->area;
  d.ks = w->k_stretch; d.ei = w->ei_bend; d.mass = w->mass; d.alpha = w->alpha; d.beta = w->beta;
  d.kernel = w->kernel;
  d.ext = w->mode;
  d.shell = w->shell;
  d.phi12 = w->shell ? 1.0 / (2.0 * (1.0 + w->poisson)) : 0.0;
  d.band_margin = w->band_margin > 0 ? w->band_margin : 2;
  d.band_cap = (int32_t)band_capacity((int64_t)band.size());
  std::vector<double> X4((size_t)np * 4, 0.0);
  for (int64_t p = 0; p < np; ++p)
    for (int a = 0; a < 3; ++a) X4[4 * p + a] = w->X0_host[3 * p + a];
  HIPCHK(c, hipMemset(F, 0, f.total));  // displacements D^n = D^{n-1} = 0, slip 0, fields 0
  HIPCHK(c, hipMemcpy(F + f.X0, X4.data(), X4.size() * 8, hipMemcpyHostToDevice));
  if (!band.empty()) HIPCHK(c, hipMemcpy(F + f.band, band.data(), band.size() * 4, hipMemcpyHostToDevice));
  HIPCHK(c, hipMemcpy(c->work + c->L.flags + d.cell0, g.flags.data(), g.ncell, hipMemcpyHostToDevice));
  HIPCHK(c, hipMemcpy(c->work + c->L.inst + k * sizeof(InstDesc), &d, sizeof d, hipMemcpyHostToDevice));
  c->wall[k].on = true;
  c->wall[k].np = np;
  c->wall[k].nband = d.nband;
  c->wall[k].band = band;
  c->wall[k].margin = w->band_margin > 0 ? w->band_margin : 2;
  c->wall[k].band_cap = band_capacity((int64_t)band.size());
  c->wall[k].X0.assign(w->X0_host, w->X0_host + 3 * np);
  c->wall[k].wss = (double*)(F + f.wss);
  c->wall[k].Xband = c->wall[k].X0;
  c->walls.clear();
  // launch grids sized for the largest band a wall may grow to (its list's
  // capacity), so that bands rebuilt on the device need no new grid
  int maxb = 0, maxmt = 0, shell = 0;
  int64_t maxp = 0;
  c->maxlines[0] = c->maxlines[1] = c->maxlines[2] = 0;
  c->maxblk = 0;
  for (int q = 0; q < c->n; ++q)
    if (c->wall[q].on) {
      const InstDesc& e = c->inst[q];
      c->walls.push_back(q);
      maxb = std::max(maxb, (int)c->wall[q].band_cap);
      maxp = std::max(maxp, c->wall[q].np);
      maxmt = std::max(maxmt, membrane_tiles(e.nth, e.nzl));
      shell |= e.shell;
      c->maxlines[0] = std::max(c->maxlines[0], e.ny * e.nz);
      c->maxlines[1] = std::max(c->maxlines[1], e.nx * e.nz);
      c->maxlines[2] = std::max(c->maxlines[2], e.nx * e.ny);
      c->maxblk = std::max(c->maxblk, (int)((e.ncell + BCELLS - 1) / BCELLS));
    }
  HIPCHK(c, hipMemcpy(c->work + c->L.walls, c->walls.data(), c->walls.size() * 4, hipMemcpyHostToDevice));
  c->dev.nwall = (int32_t)c->walls.size();
  c->dev.max_band = maxb;
  c->dev.max_np = (int32_t)maxp;
  c->dev.max_mtile = maxmt;
  c->dev.any_shell = shell;
  // default wall tile of the instance's size class (unless its shapes were
  // set): the square 256-point tile, or, on meshes too coarse for it, the
  // first smaller tile whose stencil boxes all fill at most 60 % of the
  // standard staging, so that they stay there while the wall deforms (band
  // rebuilds on the device keep the launch as it was built)
  for (SizeClass& K : c->cls) {
    if (K.shaped || std::find(K.inst.begin(), K.inst.end(), k) == K.inst.end()) continue;
    static const int pref[4][2] = {{16, 16}, {16, 8}, {8, 16}, {8, 8}};
    for (const auto& t : pref) {
      bool fits = true;
      for (int32_t i : K.inst)
        fits = fits && !(c->wall[i].on &&
                         wall_max_box(c, i, t[0], t[1]) > wall_boxcap(c->prec == 0 ? 8 : 4, t[0]) * 6 / 10);
      if (fits) {
        K.tj = t[0];
        K.tk = t[1];
        break;
      }
    }
  }
  return build_groups(c, false);
}

lbm_status lbm_set_wall(lbm_ctx* c, int32_t k, const double* X, const double* V) {
  if (!c || k < 0 || k >= c->n || !X || !V) return LBM_E_INVAL;
  if (!c->wall[k].on || !c->inst[k].ext) return fail(c, LBM_E_INVAL, "no external-solid wall at this instance");
  if (lbm_status r = inst_live(c, k)) return r;
  const InstDesc& d = c->inst[k];
  Wall& W = c->wall[k];
  const int64_t np = d.np;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  // D^n = X - X0 at the current parity, D^{n-1} = D^n - V
  std::vector<double> Dn((size_t)np * 4, 0.0), Dm((size_t)np * 4, 0.0), Dr((size_t)np * 4);
  HIPCHK(c, hipMemcpy(Dr.data(), d.Dref, (size_t)np * 32, hipMemcpyDeviceToHost));
  double moved = 0.0;
  for (int64_t p = 0; p < np; ++p)
    for (int a = 0; a < 3; ++a) {
      const double dn = X[3 * p + a] - W.X0[3 * p + a];
      Dn[4 * p + a] = dn;
      Dm[4 * p + a] = dn - V[3 * p + a];
      const double m = std::fabs(dn - Dr[4 * p + a]);
      moved = m > moved || !(m == m) ? m : moved;   // NaN propagates to the rebuild, which reports it
    }
  const int par = (int)(c->step & 1);
  HIPCHK(c, hipMemcpy(d.Xab[par], Dn.data(), (size_t)np * 32, hipMemcpyHostToDevice));
  HIPCHK(c, hipMemcpy(d.Xab[par ^ 1], Dm.data(), (size_t)np * 32, hipMemcpyHostToDevice));
  if (!(moved < (double)(W.margin - 1))) return rebuild_bands(c);
  return LBM_OK;
}

lbm_status lbm_read_wall(lbm_ctx* c, int32_t k, double* X, double* Xp, double* slip, double* Vf, double* Fp) {
  if (!c || k < 0 || k >= c->n || !c->wall[k].on) return LBM_E_INVAL;
  const InstDesc& d = c->inst[k];
  const int64_t np = d.np;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  std::vector<double> tmp((size_t)np * 4);
  auto get4 = [&](const void* src, double* dst) -> lbm_status {
    if (!dst) return LBM_OK;
    HIPCHK(c, hipMemcpy(tmp.data(), src, (size_t)np * 32, hipMemcpyDeviceToHost));
    for (int64_t p = 0; p < np; ++p)
      for (int a = 0; a < 3; ++a) dst[3 * p + a] = tmp[4 * p + a];
    return LBM_OK;
  };
  auto getr4 = [&](const void* src, double* dst) -> lbm_status {
    if (!dst) return LBM_OK;
    if (c->prec == 0) return get4(src, dst);
    std::vector<float> t((size_t)np * 4);
    HIPCHK(c, hipMemcpy(t.data(), src, (size_t)np * 16, hipMemcpyDeviceToHost));
    for (int64_t p = 0; p < np; ++p)
      for (int a = 0; a < 3; ++a) dst[3 * p + a] = t[4 * p + a];
    return LBM_OK;
  };
  int64_t tk = 0;
  lbm_status r = inst_step(c, k, &tk);
  if (r != LBM_OK) return r;
  const int par = (int)(tk & 1);
  std::vector<double> x0((size_t)np * 3);
  if ((r = get4(d.X0, x0.data())) != LBM_OK) return r;
  auto add_x0 = [&](double* dst) {
    if (dst) for (size_t q = 0; q < x0.size(); ++q) dst[q] += x0[q];
  };
  if ((r = get4(d.Xab[par], X)) != LBM_OK || (r = get4(d.Xab[par ^ 1], Xp)) != LBM_OK ||
      (r = get4(d.slip, slip)) != LBM_OK || (r = getr4(d.Vf, Vf)) != LBM_OK || (r = get4(d.Fp, Fp)) != LBM_OK)
    return r;
  add_x0(X);
  add_x0(Xp);
  return LBM_OK;
}

lbm_status lbm_wall_shear_stress(lbm_ctx* c, int32_t k, double dist, double* wss) {
  if (!c || !wss || k < 0 || k >= c->n || !c->wall[k].on) return LBM_E_INVAL;
  if (!(dist > 0.0 && dist < 64.0)) return fail(c, LBM_E_INVAL, "wall shear stress: dist outside (0, 64)");
  const InstDesc& d = c->inst[k];
  int64_t tk = 0;
  if (lbm_status r = inst_step(c, k, &tk)) return r;   // the wall's state is at the instance's step
  const double mu = (d.tau - 0.5) / 3.0;
  HIPCHK(c, launch_wss(c->dev, c->prec, (int)(tk & 1), k, d.np, dist, mu, c->wall[k].wss, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  HIPCHK(c, hipMemcpy(wss, c->wall[k].wss, (size_t)d.np * 8, hipMemcpyDeviceToHost));
  return LBM_OK;
}

lbm_status lbm_write_populations(lbm_ctx* c, int32_t k, const double* g) {
  if (!c || !g || k < 0 || k >= c->n) return LBM_E_INVAL;
  if (c->step & 1) return fail(c, LBM_E_STATE, "populations can only be written after an even number of steps");
  if (lbm_status r = inst_live(c, k)) return r;
  const Geometry& geo = c->geo[k];
  const InstDesc& d = c->inst[k];
  const int es = elem_size(c->prec);
  std::vector<char> raw((size_t)NQ * geo.ncell * es, 0);
  for (int64_t cell = 0; cell < geo.ncell; ++cell) {
    const bool fl = (geo.flags[cell] & TYPE_MASK) == T_FLUID;
    for (int i = 0; i < NQ; ++i) {
      const double v = fl ? g[(size_t)cell * NQ + i] - W[i] * d.dref : 0.0;
      char* p = raw.data() + ((size_t)i * geo.ncell + cell) * es;
      switch (c->prec) {
        case 0: std::memcpy(p, &v, 8); break;
        case 1: { float f = (float)v; std::memcpy(p, &f, 4); break; }
        case 2: { uint16_t u = f32_to_f16_rne((float)v * c->scale); std::memcpy(p, &u, 2); break; }
        default: { uint16_t u = f32_to_bf16_rne((float)v * c->scale); std::memcpy(p, &u, 2); break; }
      }
    }
  }
  HIPCHK(c, hipStreamSynchronize(c->stream));
  for (int i = 0; i < NQ; ++i)
    HIPCHK(c, hipMemcpy((char*)c->pop + ((size_t)i * c->L.NT + d.cell0) * es, raw.data() + (size_t)i * geo.ncell * es,
                        (size_t)geo.ncell * es, hipMemcpyHostToDevice));
  return LBM_OK;
}

lbm_status lbm_set_rest(lbm_ctx* c, int32_t k, double p) {
  if (!c || k < 0 || k >= c->n) return LBM_E_INVAL;
  if (c->step & 1) return fail(c, LBM_E_STATE, "rest state can only be set after an even number of steps");
  if (lbm_status r = inst_live(c, k)) return r;
  HIPCHK(c, launch_fill_rest(c->dev, c->prec, c->inst[k].cell0, c->inst[k].ncell, 3.0 * p - c->inst[k].dref,
                             c->stream));
  return LBM_OK;
}

lbm_status lbm_read_populations(lbm_ctx* c, int32_t k, double* g) {
  if (!c || !g || k < 0 || k >= c->n) return LBM_E_INVAL;
  std::vector<double> v;
  lbm_status r = read_pops(c, k, v);
  if (r != LBM_OK) return r;
  std::memcpy(g, v.data(), v.size() * 8);
  return LBM_OK;
}

lbm_status lbm_read_fields(lbm_ctx* c, int32_t k, double* p, double* u) {
  if (!c || k < 0 || k >= c->n) return LBM_E_INVAL;
  std::vector<double> v;
  lbm_status r = read_pops(c, k, v);
  if (r != LBM_OK) return r;
  const int64_t nc = c->geo[k].ncell;
  for (int64_t cell = 0; cell < nc; ++cell) {
    double s = 0, j[3] = {0, 0, 0};
    for (int i = 0; i < NQ; ++i) {
      const double g = v[(size_t)cell * NQ + i];
      s += g;
      j[0] += EXh[i] * g; j[1] += EYh[i] * g; j[2] += EZh[i] * g;
    }
    if (p) p[cell] = s / 3.0;
    if (u) for (int a = 0; a < 3; ++a) u[3 * cell + a] = j[a];
  }
  return LBM_OK;
}

lbm_status lbm_read_waveforms(lbm_ctx* c, int32_t k, double* out, int64_t cap, int64_t* n) {
  if (!c || !n || k < 0 || k >= c->n || cap < 0 || (!out && cap > 0)) return LBM_E_INVAL;
  const int64_t W = c->L.wave_cap;
  int64_t tk = 0;   // records written: the instance's own step count
  lbm_status r = inst_step(c, k, &tk);
  if (r != LBM_OK) return r;
  const int64_t have = std::min<int64_t>(tk, W);
  const int64_t cnt = std::min<int64_t>(have, cap);
  *n = cnt;
  if (cnt == 0) return LBM_OK;
  std::vector<double> ring((size_t)W * NREC);
  HIPCHK(c, hipMemcpy(ring.data(), c->work + c->L.wave + (size_t)k * W * NREC * 8, ring.size() * 8,
                      hipMemcpyDeviceToHost));
  for (int64_t q = 0; q < cnt; ++q) {
    const int64_t step = tk - cnt + q;
    std::memcpy(out + q * NREC, ring.data() + (step % W) * NREC, NREC * 8);
  }
  return LBM_OK;
}

lbm_status lbm_read_outlet_waveforms(lbm_ctx* c, int32_t k, double* out, int64_t cap, int64_t* n) {
  if (!c || !n || k < 0 || k >= c->n || cap < 0 || (!out && cap > 0)) return LBM_E_INVAL;
  const int64_t W = c->L.wave_cap;
  int64_t tk = 0;
  lbm_status r = inst_step(c, k, &tk);
  if (r != LBM_OK) return r;
  const int64_t cnt = std::min<int64_t>(std::min<int64_t>(tk, W), cap);
  *n = cnt;
  if (cnt == 0) return LBM_OK;
  std::vector<double> ring((size_t)W * NOREC);
  HIPCHK(c, hipMemcpy(ring.data(), c->work + c->L.owave + (size_t)k * W * NOREC * 8, ring.size() * 8,
                      hipMemcpyDeviceToHost));
  for (int64_t q = 0; q < cnt; ++q) {
    const int64_t step = tk - cnt + q;
    std::memcpy(out + q * NOREC, ring.data() + (step % W) * NOREC, NOREC * 8);
  }
  return LBM_OK;
}

lbm_status lbm_sync(lbm_ctx* c) {
  if (!c) return LBM_E_INVAL;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  std::vector<uint32_t> e((size_t)c->n);
  HIPCHK(c, hipMemcpy(e.data(), c->work + c->L.err, e.size() * 4, hipMemcpyDeviceToHost));
  int failed = 0, first = -1;
  for (int k = 0; k < c->n; ++k)
    if (e[k]) {
      ++failed;
      if (first < 0) first = k;
    }
  // a batch keeps running while any instance does: the failed ones are
  // frozen and reported one by one (lbm_instance_status)
  if (failed == 0 || failed < c->n) return LBM_OK;
  const std::string who = c->n > 1 ? "every instance failed; the first, " + std::to_string(first) + ": " : "";
  if (e[first] & ERR_NONFINITE) return fail(c, LBM_E_UNSTABLE, who + "boundary flux or pressure became non-finite");
  return fail(c, LBM_E_BAND, who + "a wall point left its band of cells");
}

lbm_status lbm_instance_status(lbm_ctx* c, int32_t inst) {
  if (!c) return LBM_E_INVAL;
  if (inst < 0 || inst >= c->n) return fail(c, LBM_E_INVAL, "instance index out of range");
  HIPCHK(c, hipStreamSynchronize(c->stream));
  uint32_t e = 0;
  HIPCHK(c, hipMemcpy(&e, c->work + c->L.err + (size_t)inst * 4, 4, hipMemcpyDeviceToHost));
  if (e & ERR_NONFINITE) return LBM_E_UNSTABLE;
  if (e & ERR_BAND) return LBM_E_BAND;
  return LBM_OK;
}
int64_t lbm_steps(const lbm_ctx* c) { return c ? c->step : -1; }

lbm_status lbm_set_timing(lbm_ctx* c, int32_t on) {
  if (!c) return LBM_E_INVAL;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  collect_times(c);
  for (int k = 0; k < NTIMED; ++k) { c->t_ms[k] = 0; c->t_launch[k] = 0; }
  c->timing = on != 0;
  return LBM_OK;
}

lbm_status lbm_kernel_time(lbm_ctx* c, int32_t kernel, int64_t* launches, double* ms) {
  if (!c || kernel < 0 || kernel >= NTIMED || !launches || !ms) return LBM_E_INVAL;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  collect_times(c);
  *launches = c->t_launch[kernel];
  *ms = c->t_ms[kernel];
  return LBM_OK;
}

lbm_status lbm_set_graph(lbm_ctx* c, int32_t on) {
  if (!c) return LBM_E_INVAL;
  c->use_graph = on != 0;
  return LBM_OK;
}

lbm_status lbm_set_band_check(lbm_ctx* c, int32_t every) {
  if (!c || every < 0) return LBM_E_INVAL;
  c->band_check = every;
  return LBM_OK;
}

lbm_status lbm_debug_slot_writes(lbm_ctx* c, int32_t parity, uint32_t* counts) {
  if (!c || !counts || (parity != 0 && parity != 1)) return LBM_E_INVAL;
  if (c->prec != LBM_FP32) return fail(c, LBM_E_INVAL, "the slot-write check runs on FP32 contexts");
  HIPCHK(c, hipStreamSynchronize(c->stream));
  std::vector<CTile> tiles;
  for (int i = 0; i < c->n; ++i)
    for (int64_t s0 = 0; s0 < c->inst[i].ncell; s0 += 256) tiles.push_back(CTile{i, (int32_t)s0});
  const size_t n = (size_t)NQ * (size_t)c->L.NT;
  uint32_t* cnt = nullptr;
  CTile* tab = nullptr;
  uint32_t outside = 0;   // stores past the arrays, counted after the slots
  hipError_t e = hipMalloc((void**)&cnt, (n + 1) * 4);
  if (e == hipSuccess) e = hipMalloc((void**)&tab, tiles.size() * sizeof(CTile));
  if (e == hipSuccess) e = hipMemset(cnt, 0, (n + 1) * 4);
  if (e == hipSuccess) e = hipMemcpy(tab, tiles.data(), tiles.size() * sizeof(CTile), hipMemcpyHostToDevice);
  if (e == hipSuccess) {
    Dev d = c->dev;
    d.slotcnt = cnt;
    e = launch_collide_count(d, parity, c->dev.any_nee != 0, tab, (int)tiles.size(), c->stream);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e == hipSuccess) e = hipMemcpy(counts, cnt, n * 4, hipMemcpyDeviceToHost);
  if (e == hipSuccess) e = hipMemcpy(&outside, cnt + n, 4, hipMemcpyDeviceToHost);
  if (tab) (void)hipFree(tab);
  if (cnt) (void)hipFree(cnt);
  HIPCHK(c, e);
  if (outside) return fail(c, LBM_E_STATE, "a population store outside the arrays");
  return LBM_OK;
}

lbm_status lbm_set_deterministic(lbm_ctx* c, int32_t on) {
  if (!c) return LBM_E_INVAL;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  drop_graph(c);
  c->deterministic = on != 0;
  return LBM_OK;
}

lbm_status lbm_set_overlap(lbm_ctx* c, int32_t on) {
  if (!c) return LBM_E_INVAL;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  drop_graph(c);
  c->overlap = on != 0;
  // the band-only collide pass reads the band tiles the host derives from
  // the band lists: bring them up to date
  return build_groups(c, false);
}

}  // extern "C"

// ---------------------------------------------------------------------------
// checkpoint / resume
// ---------------------------------------------------------------------------
// File: a header (magic, version, context shape, step), one record per
// instance (cells, wall points, band size), then the raw device state in a
// fixed order: populations, cell flags (band bits), 0D boundary records,
// per-instance step counters, waveform rings, inlet snapshots, error and
// motion words, and per wall its displacements D^n / D^{n-1}, slip
// integral, last interpolated velocity and force, displacement at the last
// band build and the band cell list.  Band velocities and forces are not
// saved: every step recomputes them before use.

namespace {

constexpr char CKPT_MAGIC[8] = {'L', 'B', 'M', '0', 'D', '3', 'D', 'C'};
constexpr uint32_t CKPT_VERSION = 5;

struct CkptHeader {
  char magic[8];
  uint32_t version;
  int32_t n, prec, wave_cap;
  int64_t NT, nv0, step;
  float scale;
  uint32_t pad;
};

struct CkptInst {
  int64_t ncell, np;
  int32_t has_wall, nband, margin, pad;
};

// the pieces of device state a checkpoint holds, in file order
std::vector<std::pair<char*, size_t>> ckpt_pieces(lbm_ctx* c) {
  std::vector<std::pair<char*, size_t>> v;
  const size_t n = (size_t)c->n;
  v.push_back({(char*)c->pop, (size_t)NQ * c->L.NT * elem_size(c->prec)});
  v.push_back({c->work + c->L.flags, (size_t)c->L.NT});
  v.push_back({c->work + c->L.bc, NBC * n * sizeof(BcDev)});
  v.push_back({c->work + c->L.st, n * sizeof(InstState)});
  v.push_back({c->work + c->L.wave, n * (size_t)c->L.wave_cap * NREC * 8});
  v.push_back({c->work + c->L.owave, n * (size_t)c->L.wave_cap * NOREC * 8});
  v.push_back({c->work + c->L.v0, (size_t)c->L.nv0 * r4_size(c->prec)});
  v.push_back({c->work + c->L.err, n * 4});
  v.push_back({c->work + c->L.moved, 4});
  for (int k = 0; k < c->n; ++k) {
    if (!c->wall[k].on) continue;
    const InstDesc& d = c->inst[k];
    const size_t np = (size_t)d.np;
    v.push_back({(char*)d.Xab[0], np * 32});
    v.push_back({(char*)d.Xab[1], np * 32});
    v.push_back({(char*)d.slip, np * 32});
    v.push_back({(char*)d.Vf, np * r4_size(c->prec)});
    v.push_back({(char*)d.Fp, np * 32});
    v.push_back({(char*)d.Dref, np * 32});
  }
  return v;
}

}  // namespace

extern "C" {

lbm_status lbm_save(lbm_ctx* c, const char* path) {
  if (!c || !path) return LBM_E_INVAL;
  if (lbm_status r = refresh_bands(c)) return r;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  FILE* f = std::fopen(path, "wb");
  if (!f) return fail(c, LBM_E_INVAL, std::string("cannot open checkpoint file for writing: ") + path);
  bool ok = true;
  auto put = [&](const void* p, size_t b) { ok = ok && std::fwrite(p, 1, b, f) == b; };
  CkptHeader h;
  std::memset(&h, 0, sizeof h);
  std::memcpy(h.magic, CKPT_MAGIC, 8);
  h.version = CKPT_VERSION;
  h.n = c->n; h.prec = c->prec; h.wave_cap = c->L.wave_cap;
  h.NT = c->L.NT; h.nv0 = c->L.nv0; h.step = c->step; h.scale = c->scale;
  put(&h, sizeof h);
  for (int k = 0; k < c->n; ++k) {
    CkptInst r;
    std::memset(&r, 0, sizeof r);
    r.ncell = c->geo[k].ncell;
    r.has_wall = c->wall[k].on ? 1 : 0;
    r.np = c->wall[k].on ? c->wall[k].np : 0;
    r.nband = c->wall[k].on ? c->wall[k].nband : 0;
    r.margin = c->wall[k].margin;
    put(&r, sizeof r);
  }
  std::vector<char> buf;
  for (const auto& pc : ckpt_pieces(c)) {
    buf.resize(pc.second);
    const hipError_t e = hipMemcpy(buf.data(), pc.first, pc.second, hipMemcpyDeviceToHost);
    if (e != hipSuccess) {
      std::fclose(f);
      return fail(c, LBM_E_DEVICE, std::string("checkpoint read-back: ") + hipGetErrorString(e));
    }
    put(buf.data(), pc.second);
  }
  for (int k = 0; k < c->n; ++k)
    if (c->wall[k].on) put(c->wall[k].band.data(), c->wall[k].band.size() * 4);
  ok = (std::fclose(f) == 0) && ok;
  if (!ok) return fail(c, LBM_E_INVAL, std::string("checkpoint write failed: ") + path);
  return LBM_OK;
}

lbm_status lbm_load(lbm_ctx* c, const char* path) {
  if (!c || !path) return LBM_E_INVAL;
  FILE* f = std::fopen(path, "rb");
  if (!f) return fail(c, LBM_E_INVAL, std::string("cannot open checkpoint file: ") + path);
  // The whole file is read and checked on the host before anything reaches
  // the device, so a truncated or corrupt file leaves the context untouched.
  bool ok = true;
  auto get = [&](void* p, size_t b) { ok = ok && std::fread(p, 1, b, f) == b; };
  auto bad = [&](const std::string& m) {
    if (f) std::fclose(f);
    f = nullptr;
    return fail(c, LBM_E_STATE, "checkpoint does not fit this context: " + m);
  };
  CkptHeader h;
  get(&h, sizeof h);
  if (!ok || std::memcmp(h.magic, CKPT_MAGIC, 8) != 0 || h.version != CKPT_VERSION) return bad("not a checkpoint");
  if (h.n != c->n || h.prec != c->prec || h.wave_cap != c->L.wave_cap || h.NT != c->L.NT || h.nv0 != c->L.nv0 ||
      h.scale != c->scale)
    return bad("instances, precision, storage scale or waveform capacity differ");
  if (h.step < 0) return bad("negative step count");
  std::vector<CkptInst> r((size_t)c->n);
  for (int k = 0; k < c->n; ++k) {
    get(&r[k], sizeof r[k]);
    if (!ok) return bad("truncated");
    const bool wall = c->wall[k].on;
    if (r[k].ncell != c->geo[k].ncell || r[k].has_wall != (wall ? 1 : 0) || (wall && r[k].np != c->wall[k].np))
      return bad("an instance's cells or wall differ");
    if (wall && (r[k].nband < 0 || r[k].nband > c->wall[k].band_cap))
      return bad("a saved band is negative or exceeds the wall buffer's capacity");
    if (wall && (r[k].margin < 1 || r[k].margin > 64)) return bad("a saved band margin is outside [1, 64]");
  }
  const auto pieces = ckpt_pieces(c);
  std::vector<std::vector<char>> data(pieces.size());
  for (size_t q = 0; q < pieces.size(); ++q) {
    data[q].resize(pieces[q].second);
    get(data[q].data(), pieces[q].second);
    if (!ok) return bad("truncated");
  }
  std::vector<std::vector<int32_t>> bands((size_t)c->n);
  for (int k = 0; k < c->n; ++k) {
    if (!c->wall[k].on) continue;
    bands[k].resize((size_t)r[k].nband);
    get(bands[k].data(), bands[k].size() * 4);
    if (!ok) return bad("truncated");
  }
  char extra;
  if (std::fread(&extra, 1, 1, f) != 0) return bad("trailing bytes after the band lists");
  std::fclose(f);
  f = nullptr;

  // pieces 1..3 are the flags, the 0D records and the step counters; 7 the
  // error words
  const uint8_t* fl = (const uint8_t*)data[1].data();
  const BcDev* bc = (const BcDev*)data[2].data();
  const InstState* st = (const InstState*)data[3].data();
  const uint32_t* ew = (const uint32_t*)data[7].data();
  for (int k = 0; k < c->n; ++k) {
    if (ew[k] & ~(ERR_NONFINITE | ERR_BAND | ERR_FROZEN)) return bad("an error word is malformed");
    const Geometry& g = c->geo[k];
    const InstDesc& d = c->inst[k];
    // cell types and the near bits are fixed by the geometry: only the band
    // bit may differ from the context's own flags
    int64_t nbandbits = 0;
    for (int64_t lc = 0; lc < g.ncell; ++lc) {
      const uint8_t a = fl[d.cell0 + lc], b = g.flags[(size_t)lc];
      if ((a & (uint8_t)~F_BAND) != (b & (uint8_t)~F_BAND)) return bad("cell types differ from the context's geometry");
      if (a & F_BAND) {
        if ((a & TYPE_MASK) != T_FLUID) return bad("a band bit on a non-FLUID cell");
        ++nbandbits;
      }
    }
    for (int b = 0; b < NBC; ++b) {
      const BcDev& q = bc[NBC * k + b];
      if (q.boundary != b || q.kind < BC_PRESSURE || q.kind > BC_LV || (q.kind == BC_LV && b != 0) ||
          (q.vmode != 0 && q.vmode != 1) || q.vkind < VK_CONST || q.vkind > VK_SNAPSHOT)
        return bad("a 0D boundary record is malformed");
    }
    if (st[k].counter != 0u || st[k].step < 0) return bad("an instance's step record is malformed");
    if (!c->wall[k].on) {
      if (nbandbits != 0) return bad("band bits in an instance without a wall");
      continue;
    }
    // band: ascending local FLUID cells, exactly those with the band bit
    const std::vector<int32_t>& band = bands[k];
    if ((int64_t)band.size() != nbandbits) return bad("the band list and the band bits disagree");
    for (size_t q = 0; q < band.size(); ++q) {
      if (band[q] < 0 || band[q] >= g.ncell || (q > 0 && band[q] <= band[q - 1]))
        return bad("band cells out of range or not ascending");
      if (!(fl[d.cell0 + band[q]] & F_BAND)) return bad("a band cell without its band bit");
    }
  }

  // everything checked: upload
  HIPCHK(c, hipStreamSynchronize(c->stream));
  drop_graph(c);
  for (size_t q = 0; q < pieces.size(); ++q)
    if (pieces[q].second)
      HIPCHK(c, hipMemcpy(pieces[q].first, data[q].data(), pieces[q].second, hipMemcpyHostToDevice));
  int maxb = 0;
  for (int k = 0; k < c->n; ++k) {
    Geometry& g = c->geo[k];
    InstDesc& d = c->inst[k];
    std::memcpy(g.flags.data(), fl + d.cell0, (size_t)g.ncell);
    if (!c->wall[k].on) continue;
    Wall& W = c->wall[k];
    std::vector<int32_t>& band = bands[k];
    if (!band.empty()) HIPCHK(c, hipMemcpy(d.band, band.data(), band.size() * 4, hipMemcpyHostToDevice));
    d.nband = r[k].nband;
    d.band_margin = r[k].margin;
    HIPCHK(c, hipMemcpy(c->work + c->L.inst + k * sizeof(InstDesc), &d, sizeof d, hipMemcpyHostToDevice));
    W.band.swap(band);
    W.nband = d.nband;
    W.margin = r[k].margin;
    // positions the restored band was built around: X0 + Dref
    std::vector<double> Dr((size_t)d.np * 4);
    HIPCHK(c, hipMemcpy(Dr.data(), d.Dref, (size_t)d.np * 32, hipMemcpyDeviceToHost));
    W.Xband.resize((size_t)d.np * 3);
    for (int64_t p = 0; p < d.np; ++p)
      for (int a = 0; a < 3; ++a) W.Xband[3 * p + a] = W.X0[3 * p + a] + Dr[4 * p + a];
    maxb = std::max(maxb, W.nband);
  }
  (void)maxb;
  c->bands_stale = false;
  c->step = h.step;
  return build_groups(c, false);
}

const char* lbm_last_error(const lbm_ctx* c) { return c ? c->err.c_str() : g_init_err.c_str(); }

void lbm_destroy(lbm_ctx* c) {
  if (!c) return;
  (void)hipStreamSynchronize(c->stream);
  if (c->side) (void)hipStreamSynchronize(c->side);
  collect_times(c);
  for (auto& p : c->pool) {
    (void)hipEventDestroy(p.a);
    (void)hipEventDestroy(p.b);
  }
  drop_graph(c);
  for (hipEvent_t e : {c->ev_fork, c->ev_wall, c->ev_join, c->ev_red})
    if (e) (void)hipEventDestroy(e);
  if (c->side) (void)hipStreamDestroy(c->side);
  delete c;
}

int64_t lbm_num_cells(const lbm_ctx* c, int32_t k) {
  if (!c || k < 0 || k >= c->n) return -1;
  return c->geo[k].ncell;
}

int32_t lbm_bytes_per_population(const lbm_ctx* c) { return c ? elem_size(c->prec) : -1; }

}  // extern "C"
