// lbm_internal.h -- device-side data layout of the gfx950 library (private).
//
// One context holds n instances (n = 1 for a single box).  Every per-cell
// array is concatenated over the instances; the populations are one
// structure-of-arrays block A[19][NT] (NT = total cells), updated in place with
// the AA pattern: an even step reads and writes a cell's own slots (writing
// direction i into slot opp(i)), an odd step reads from and writes to the
// neighbours.  Everything a kernel needs about an instance sits in its
// InstDesc, found from the block index through a block->instance table.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbm {

constexpr int NQ = 19;
constexpr int NREC = 14;          // doubles per waveform record
constexpr int MIN_TILE = 128;     // smallest collide tile (workgroup 128, 1 cell per lane)
constexpr int RBLOCK = 256;       // boundary-reduction workgroup
constexpr int RCHUNK = 256;       // layer cells per reduction workgroup (one per lane)
constexpr int WBLOCK = 256;       // wall / band workgroups

// Outlets: the OUTLET ghosts of an instance may form up to NOUT separate
// outlets, each with its own 0D model; an OUTLET ghost's cell-type byte
// carries its outlet index k in bits 5-7.  0D records per instance (NBC):
// 0 inlet, 1 outlet 0, 2 exterior, 2 + k outlet k >= 1.  Boundary layers
// per instance (NPL): 0 inlet, 1 outlet 0, 2 mid-length plane, 2 + k outlet k.
constexpr int NOUT = 8;
constexpr int NBC = 2 + NOUT;
constexpr int NPL = 2 + NOUT;
constexpr int OUT_SHIFT = 5;
__host__ __device__ constexpr int outlet_slot(int k) { return k == 0 ? 1 : 2 + k; }
constexpr int NOREC = 3 * NOUT;   // per-outlet record: flux, mean gauge pressure, Pw

enum : uint8_t { T_FLUID = 0, T_SOLID = 1, T_INLET = 2, T_OUTLET = 3, T_EXTP = 4 };
constexpr uint8_t TYPE_MASK = 7;
constexpr uint8_t F_NEAR = 8;     // FLUID cell with at least one non-FLUID neighbour
constexpr uint8_t F_BAND = 16;    // FLUID cell inside a wall's band (may carry force)

enum : int32_t { BC_PRESSURE = 0, BC_VELOCITY = 1, BC_WK3 = 2, BC_LV = 3 };
enum : int32_t { VK_CONST = 0, VK_CORRECT = 1, VK_SNAPSHOT = 2 };

// Error word of an instance: what failed (NONFINITE, BAND), and FROZEN once
// the instance is no longer stepped.  The first reduction of the step after
// a failure sets FROZEN (so the failing step itself runs to its end and the
// frozen state sits at the instance's own step count); a band rebuild that
// fails on the host sets both at once, between steps.
enum : uint32_t { ERR_NONFINITE = 1u, ERR_BAND = 2u, ERR_FROZEN = 4u };

// 0D boundary model: configuration, state, and what it hands the collide
// kernel for the current step.
struct BcDev {
  int32_t kind, boundary;
  double par[16];
  double area;             // layer cells (flux -> mean velocity)
  // state
  double Pw, Pv;
  int64_t Td, cycle;
  int32_t open;
  int32_t inflow;          // inflow seen since the valve opened (LV)
  // output of the last update (valid for the step being taken)
  int32_t vmode;           // 0 pressure type, 1 velocity type
  int32_t vkind;           // VK_*
  int32_t snap;            // 1 on the step the valve closes
  double pstar;            // gauge P*
  double dstar;            // 3 P* (shifted density target)
  double vz;               // constant axial v*, or the axial correction dv
  double S;                // smoothing factor (LV)
};

struct InstDesc {
  int32_t nx, ny, nz;
  int32_t red0, nred;      // reduction blocks
  int32_t lay_off[NPL], lay_n[NPL];   // boundary-layer lists (planes as above) in the lay array
  int64_t cell0, ncell;
  int64_t v0_off;          // first entry of this instance's inlet snapshot (nx*ny)
  double tau;
  double omega;            // 1 / tau
  double dref;             // 3 p_ref: stored populations are g - w_i dref
  // wall (has_wall = 0: none)
  int32_t has_wall, nth, nzl, nband;
  int32_t kernel;          // delta kernel: 0 Peskin 4-point, 1 cosine 4-point
  int32_t ext;             // 1: external solid (points moved by the caller)
  int32_t shell;           // 1: off-diagonal terms of the wall model (shear, mixed bending)
  int32_t nee;             // 1: normal-neighbour x_f in the extrapolation at ghosts
  int64_t np;
  void* u4;                // R4 per local cell: unforced velocity (band cells)
  void* b4;                // R4 per local cell: IB force density (band cells)
  double* X0;              // double4 per point
  double* Xab[2];          // double4 per point, ping-pong D^n / D^{n-1}, D = X - X0
  double* slip;            // double4 per point
  void* Vf;                // R4 per point (last step, for read-back)
  void* Fp;                // double4 per point: penalty force on the fluid (last step)
  int32_t* band;           // local cell ids of the band
  int32_t band_margin;     // cells kept around the stencils (band rebuild)
  int32_t band_cap;        // capacity of the band list
  int64_t cblk0;           // first block count of this instance (band rebuild)
  double* Dref;            // double4 per point: displacement when the band was built
  double ds_th, ds_z, area, ks, ei, mass, alpha, beta;
  double phi12;            // 1 / (2 (1 + Poisson's ratio)), shell model
};

struct InstState {
  int64_t step;
  uint32_t counter;        // finished reduction blocks of the current step
  uint32_t pad;
};

struct RedTab {
  int32_t inst, plane, start, count;
};

// Everything a launch needs (passed by value as the kernel argument).
struct Dev {
  void* pop;
  int64_t NT;
  float scale, inv_scale;          // 16-bit storage scale
  const uint8_t* flags;
  const uint64_t* nbr;             // per NEAR cell: type of c - e_i in bits 3i..3i+2 (i = 1..18);
                                   // 16-bit storage only
  const InstDesc* inst;
  const int32_t* lay;              // layer cell lists (local cell ids)
  const RedTab* red;
  double* red_part;                // 2 doubles per reduction block
  BcDev* bc;                       // NBC per instance
  InstState* st;
  double* wave;                    // [inst][wave_cap][NREC]
  double* owave;                   // [inst][wave_cap][NOREC]: per outlet Q, p, Pw
  int32_t wave_cap;
  int32_t nwall;
  void* v0;                        // R4 per snapshot entry
  uint32_t* err;                   // per instance: ERR_* bits
  uint32_t* moved;                 // max wall motion since the band was built (float bits)
  // band rebuild on the device: cell marks (two byte arrays over all cells),
  // band cells per block of BCELLS cells, and the gate word (1: rebuild now)
  uint32_t* slotcnt;   // slot-writer check only: 19 * NT store counts (else null)
  uint8_t* bmark;
  uint8_t* btmp;
  int32_t* bcnt;
  uint32_t* gate;
  const int32_t* walls;            // instance ids with a wall
  int32_t max_band, max_np;
  int32_t any_nee;                 // some instance uses the normal-neighbour extrapolation
  int32_t max_mtile;               // largest membrane tile count of a wall (membrane_tiles)
  int32_t any_shell;               // some wall takes the shell model's off-diagonal terms
};

// membrane step tiles: MEM_TJ x MEM_TK points (theta x z) per workgroup
constexpr int MEM_TJ = 64, MEM_TK = WBLOCK / MEM_TJ;
inline int membrane_tiles(int nth, int nzl) { return ((nth + MEM_TJ - 1) / MEM_TJ) * ((nzl + MEM_TK - 1) / MEM_TK); }

// collide tile: BS * CPT consecutive local cells of one instance
struct CTile {
  int32_t inst;
  int32_t start;
};

}  // namespace lbm

// launchers (lbm_kernels.hip)
namespace lbm {
hipError_t launch_reduce(const Dev& d, int prec, int parity, int nred, hipStream_t s);
// collide-stream over a size class: ntile tiles of the table tab, workgroup
// size bs (128, 256, 512) and cpt (1, 2) cells per lane; nee: the build with
// the normal-neighbour extrapolation (for tiles next to a 0D ghost of an
// instance that asks for it); mode selects all fluid cells, those outside
// the wall band, or the band cells only
enum { COLLIDE_ALL = 0, COLLIDE_BULK = 1, COLLIDE_BAND = 2 };
hipError_t launch_collide(const Dev& d, int prec, int parity, int bs, int cpt, bool nee, const CTile* tab,
                          int ntile, int mode, hipStream_t s);
hipError_t launch_band(const Dev& d, int prec, int parity, hipStream_t s);
// the slot-writer check: the FP32 collide counting its stores (d.slotcnt)
// over tiles of 256 cells
hipError_t launch_collide_count(const Dev& d, int parity, bool nee, const CTile* tab, int ntile, hipStream_t s);
// the boundary reductions and the band moments in one launch
hipError_t launch_reduce_band(const Dev& d, int prec, int parity, int nred, hipStream_t s);
// LDS staging capacity of a wall tile's stencil box (cells), standard and
// large-box kernels; element size 8 (FP64) or 4 (FP32 velocities)
constexpr int wall_boxcap(int elem, int tj) { return elem == 8 ? 1024 : (tj == 32 ? 2048 : 1792); }
constexpr int wall_boxcap_big(int elem) { return elem == 8 ? 2560 : 4096; }
// wall exchange over the walls of a size class, tiles of tj x tk points
// (8 x 32, 16 x 16, 32 x 8, 8 x 16, 16 x 8, 8 x 8); tiles = tile count of the
// class's largest wall; colour >= 0 takes only the tiles of that colour
// (WALL_COLOURS classes, tiles of one colour two tiles apart in theta and in z)
constexpr int WALL_COLOURS = 6;
hipError_t launch_wall(const Dev& d, int prec, int parity, int tj, int tk, bool big, const int32_t* walls, int nwall,
                       int tiles, int colour, hipStream_t s);
// Band rebuild on the device: the gate opens once the motion word reaches
// thresh; then every wall's band is rebuilt around the current positions
// (parity) by marking the stencil bases, dilating the marks along x, y and
// z, setting the band bits of the flags and compacting the band list.
// maxlines: most lines along x, y, z of a walled instance; maxblk: most
// blocks of BCELLS cells of one.
constexpr int BCELLS = 1024;
hipError_t launch_band_rebuild(const Dev& d, int parity, float thresh, const int maxlines[3], int maxblk,
                               hipStream_t s);
// wall shear stress of the np points of instance inst's wall into out (np
// doubles, device): fluid velocity at dist along the inward normal, mu the
// dynamic viscosity
hipError_t launch_wss(const Dev& d, int prec, int parity, int inst, int64_t np, double dist, double mu, double* out,
                      hipStream_t s);
// wall motion since the band was built, into the moved word (parity: the
// current displacement's half of the ping-pong pair)
hipError_t launch_motion(const Dev& d, int parity, hipStream_t s);
hipError_t launch_membrane(const Dev& d, int parity, hipStream_t s);
hipError_t launch_fill_rest(const Dev& d, int prec, int64_t cell0, int64_t ncell, double dshift, hipStream_t s);
}  // namespace lbm
