// lattice.hip -- C-ABI runtime of the lattice field step (see include/lattice.h).
//
// The runtime turns a call lattice_step(n) into a schedule of stencil passes
// (one pass per kick point) and launches them on the context stream:
//   leapfrog   pass k: kick (half after a sync, else full) then local drift
//   VV2 / VV4  kick points p = 0..M of the sub-step sequence (M = n or 3n);
//              pass p: drift that ends at p (on load), kick h_{p-1}/2, sample
//              energies, kick h_p/2.  The two half kicks that meet at an inner
//              point share one force evaluation.
// For a fixed or absent background every coefficient is known beforehand and
// uploaded as a table; for self-consistent expansion the pass that samples the
// energies at point p also advances (a, b) and writes the next pass's drift and
// kick coefficients on the device, so no host round trip sits between passes.
#include <hip/hip_runtime.h>
#include <hipfft/hipfft.h>

#include <algorithm>
#include <cmath>
#include <cstddef>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <type_traits>
#include <utility>
#include <vector>

#include "lattice.h"
#include "common.hpp"
#include "stage_scalar.hpp"
#include "stage_rows.hpp"
#include "stage_u1.hpp"
#include "stage_su2.hpp"
#include "stage_gauss.hpp"
#include "stage_adjoint.hpp"
#include "stage_batch.hpp"
#include "stage_slab.hpp"
#include "spectrum.hpp"
#include "stage_adjoint_self.hpp"

using namespace lat;

// Fixed device scratch of lattice_energy_noalloc: every GPU the library runs
// on holds one copy (513 KiB) until the process ends.  Host code never uses
// this name as an address; it uses the per-device pointer that
// hipGetSymbolAddress returns for it.
static __device__ __align__(256) unsigned char scratch[512 * 1024 + 1024];

struct lat_ctx;

namespace {

thread_local std::string g_init_error;

// U(1) sector (defined at the end of this file)
lat_status u1_step_lf(lat_ctx *c, int64_t ns, int dir);
lat_status u1_sync(lat_ctx *c);
lat_status u1_energy(lat_ctx *c, lat_energies *out);
lat_status su2_step_lf(lat_ctx *c, int64_t ns, int dir);
lat_status gauge_step_vv(lat_ctx *c, int64_t ns, int dir);
lat_status su2_sync(lat_ctx *c);
lat_status su2_energy(lat_ctx *c, lat_energies *out);
size_t su2_partial_capacity(int N);
int su2_zc(int N, bool band);
void su2_geometry(lat_ctx *c);
size_t u1_partial_capacity(int N);
void u1_geometry(lat_ctx *c);
lat_status batch_step(lat_ctx *c, int64_t nsteps);

struct TileCfg {
    int tx, ty;
};
constexpr TileCfg kTiles[] = {{64, 4}, {64, 8}, {32, 8}, {16, 16}, {8, 8}};
constexpr int kNumTiles = sizeof(kTiles) / sizeof(kTiles[0]);

enum Variant : int {
    kKickOnly = 0,     // no drift, kick, momenta in place (VV first point, LF sync)
    kKickOnlyRed = 1,  // same + reductions (self-consistent first point)
    kDriftKick = 2,    // drift on load, kick (VV inner and last points)
    kDriftKickRed = 3, // same + reductions (self-consistent)
    kKickDrift = 4,    // kick, drift at end (leapfrog)
    kEnergy = 5        // kick on a copy + reductions, writes nothing
};

}  // namespace

struct lat_ctx {
    lat_params p{};
    hipStream_t stream = nullptr;
    int device = 0;
    bool f32 = false;
    bool u1 = false;
    bool su2 = false;
    int nf = 1;
    int N = 0;
    size_t vol = 0;
    size_t esize = 8;
    // field arrays: [0] = caller's buffer, [1] = library shadow
    void *phi[2][2] = {};
    void *pi[2][2] = {};
    int cur_phi[2] = {0, 0};
    int cur_pi[2] = {0, 0};
    void *A[3][2] = {};
    void *piA[3] = {};
    int cur_A[3] = {0, 0, 0};
    // SU(2): doublet components and links ([0] caller's, [1] shadow), momenta in place;
    // one buffer parity for all of them
    void *dbl[4][2] = {};
    void *dpi[4] = {};
    void *lnk[12][2] = {};
    void *efl[9] = {};
    int cur_su2 = 0;
    int su2_zc = 1;
    int su2_band = 0;   // y tiles per XCD band of the SU(2) block order (0: plane-wide order)
    int su2_nt = 1;     // step passes stream the momenta and output records non-temporally
    // per-site records of the doublet and links while lattice_step runs (ping-pong)
    double4 *su2_aos[2] = {};
    int su2_aos_on = 0;
    bool u1_rows = false;   // whole-row U(1) leapfrog kernel
    int u1_ty = 4, u1_zc = 8;
    int u1_ezc = 1;         // z planes per block of the U(1) energy pass
    // scratch
    double *partials = nullptr;
    size_t partial_cap = 0;
    unsigned *ticket = nullptr;
    ScaleRecord *sc = nullptr;
    ScaleRecord *sc_host = nullptr;
    PassCoef *coef = nullptr;
    size_t coef_cap = 0;
    // pinned staging for the table: a ring of slots, so the host fills the next
    // call's table while earlier uploads are still queued behind running passes
    static constexpr int kRing = 4;
    PassCoef *coef_host = nullptr;      // the current slot
    PassCoef *ring_base = nullptr;
    size_t ring_cap = 0;                // entries per slot
    int ring_slot = 0;
    hipEvent_t ring_ev[kRing] = {};
    bool ring_pending[kRing] = {};
    // host mirror of the clock
    double t = 0.0;
    int lf_stag = 0;
    int64_t step = 0;
    // launch geometry
    int tile = 0;
    bool rows = false;   // whole-row kernel (N = 64 * XS)
    int rows_ty = 8;
    int rows_pf = 1;     // whole-row kernel prefetch depth (planes)
    int en_pf = 0, en_zc = 0, en_ty = 0, en_nblocks = 0;   // energy pass geometry (en_nblocks 0: the stage passes')
    int rows_vw = 1;     // whole-row kernel sites per lane and access (1, or 16-byte vectors)
    int rows_y_fastest = 0;   // whole-row kernel block order (see stage_rows.hpp)
    int rows_alternate = 0;   // whole-row kernel: alternate the z march direction pass by pass
    int rows_lp = 0;          // whole-row kernel store policy (see launch_rows)
    int rows_split = 6;       // store policy 1: eighths of the march with non-temporal stores
    int rows_zpair = 0;       // whole-row kernel: odd z chunks march the other way
    int zc = 0;
    int tiles_x = 0, tiles_y = 0, chunks_z = 0, nblocks = 0;
    // launch statistics and optional event timing
    int64_t launches[8] = {};
    double kernel_ms[8] = {};
    bool profiling = false;
    struct Timed {
        hipEvent_t start, stop;
        int kind;
    };
    std::vector<Timed> timed;      // recorded, not yet harvested
    std::vector<hipEvent_t> spare; // reusable events
    // adjoint scratch: lphi, lpi per field, two buffers each; checkpoints; partials
    void *lam[2][2][2] = {};       // [kind 0 = lphi, 1 = lpi][field][buffer]
    int cur_lam[2][2] = {};
    double *ckpt = nullptr;
    size_t ckpt_count = 0;
    double *adj_partials = nullptr;
    size_t adj_partial_cap = 0;
    double *self_seg = nullptr;         // self-consistent adjoint: the states of one segment
    size_t self_seg_cap = 0;            // (in states)
    double *self_part = nullptr;        // its per-block partials and totals
    size_t self_part_cap = 0;
    bool sums_fresh = false;            // sc->sums are those of the current state (see lattice_energy)
    int slab_steps = 0, slab_zs = 0, slab_yb = 0;   // lf_slab: steps per launch (0: off), planes and rows per block
    const void *slab_fn = nullptr;      // the lf_slab instance for those, and its dynamic LDS
    size_t slab_lds = 0;
    double *traj_rec = nullptr;         // set: velocity-Verlet passes store (a, b) of kick point p at traj_rec + 2 p
    double *self_traj = nullptr;        // a, a' of every step, scale records of the checkpoints, scalars
    size_t self_traj_cap = 0;           // (in doubles)
    // batch of independent lattices
    bool batch = false;
    std::vector<lat_ctx *> subs;
    void *reals_dev = nullptr;          // BatchReal<T>[n]
    std::vector<char> reals_host;       // host copy (bytes)
    int2 *block_work = nullptr;         // BatchArgs::block_work table
    std::vector<int2 *> seg_work;       // per step segment: its block table
    std::vector<int> seg_blocks;
    int batch_blocks = 0;
    std::vector<void *> pi_scratch;
    std::map<int, std::pair<int, int>> batch_tile;   // N -> (tile x, z chunk)
    int batch_parity = 0;
    hipStream_t capture_stream = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    hipGraph_t graph = nullptr;
    int64_t graph_n = 0;
    int graph_parity = -1;
    // single-lattice graphs of the pass launches of lattice_step calls, keyed
    // by (signed step count, leapfrog phase); least recently used is replaced
    struct StepGraph {
        hipGraphExec_t exec = nullptr;
        int64_t n = 0;
        int stag = 0;
        int end_phi[2] = {0, 0}, end_pi[2] = {0, 0};
        int64_t launches[8] = {};
        uint64_t used = 0;
    };
    static constexpr int kStepGraphs = 4;
    StepGraph sg[kStepGraphs];
    uint64_t sg_clock = 0;
    // power spectra (allocated on first use)
    hipfftHandle fft_plan = nullptr;      // float64 real-to-complex, N^3
    hipfftHandle fft_inv = nullptr;       // float64 complex-to-real, N^3 (adjoint seed)
    double *fft_in = nullptr;
    double2 *fft_out = nullptr;
    double2 *fft_out2 = nullptr;          // second half spectrum (occupation number: momenta)
    double *spec_part = nullptr;        // per-block sums and counts, then the per-bin totals
    std::string err;
};

namespace {

lat_status fail(lat_ctx *c, lat_status s, const std::string &msg)
{
    if (c) c->err = msg;
    else g_init_error = msg;
    return s;
}

#define HIPCHK(ctx, expr)                                                                 \
    do {                                                                                  \
        hipError_t e_ = (expr);                                                           \
        if (e_ != hipSuccess)                                                             \
            return fail(ctx, LAT_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

// ---------------------------------------------------------------------------
// background closed form (eq. ScaleFactorPowerLaw)
// ---------------------------------------------------------------------------
void fixed_ab(const lat_params &p, double t, double *a, double *b)
{
    const double pw = 2.0 / (3.0 * (1.0 + p.w_eos) - 2.0 * p.alpha);
    const double u = 1.0 + p.H0 * (t - p.t_ref) / pw;
    *a = p.a0 * std::pow(u, pw);
    *b = p.a0 * p.H0 * std::pow(u, pw - 1.0);
}

double scale_at(const lat_ctx *c, double t)
{
    if (c->p.expansion == LAT_EXP_FIXED) {
        double a, b;
        fixed_ab(c->p, t, &a, &b);
        return a;
    }
    return 1.0;
}

// ---------------------------------------------------------------------------
// launch geometry
// ---------------------------------------------------------------------------
int pick_tile(int N)
{
    if (N % 64 == 0 && N >= 128) return 1;   // 64 x 8
    if (N % 64 == 0) return 0;               // 64 x 4
    if (N % 32 == 0) return 2;               // 32 x 8
    if (N % 16 == 0) return 3;               // 16 x 16
    return 4;                                // 8 x 8
}

bool rows_ok(int N) { return N == 64 || N == 128 || N == 256; }

// z chunk giving about `target` blocks; down to one plane per block for small
// lattices, where a longer march is a serial chain over too few blocks
// (32^3 single field: 4.2 against 5.4 us per step with chunks of 4)
int auto_chunk(int N, long xy_blocks, long target)
{
    long z = (long)N * xy_blocks / target;
    if (z < 1) z = 1;
    if (z > N) z = N;
    return (int)z;
}

void set_geometry(lat_ctx *c, int tile, int zc)
{
    const int N = c->N;
    c->rows = false;
    c->tile = tile;
    c->tiles_x = (N + kTiles[tile].tx - 1) / kTiles[tile].tx;
    c->tiles_y = (N + kTiles[tile].ty - 1) / kTiles[tile].ty;
    if (zc <= 0) zc = auto_chunk(N, (long)c->tiles_x * c->tiles_y, 512);
    if (zc > N) zc = N;
    c->zc = zc;
    c->chunks_z = (N + zc - 1) / zc;
    c->nblocks = c->tiles_x * c->tiles_y * c->chunks_z;
}

void set_rows_geometry(lat_ctx *c, int ty, int zc)
{
    const int N = c->N;
    c->rows = true;
    c->rows_ty = ty;
    c->tiles_x = 1;
    c->tiles_y = (N + ty - 1) / ty;
    if (zc <= 0) zc = auto_chunk(N, c->tiles_y, 256);
    if (zc > N) zc = N;
    c->zc = zc;
    c->chunks_z = (N + zc - 1) / zc;
    c->nblocks = c->tiles_y * c->chunks_z;
}

// Energy pass geometry of the whole-row kernel.  Read-only, the pass needs
// more bytes in flight than the stage passes' one wave per SIMD give: at
// N = 256 it runs 32-plane z chunks with two waves per SIMD, in float64 one
// plane ahead in 8-row blocks (235 VGPRs; 108-113 against 124-130 us with
// 4-row blocks and 134-144 us in the stage geometry), in float32 two planes
// ahead in 4-row blocks (56-58 against 74-75 us).  LATTICE_ENERGY_GEOM=
// "pf,zc[,ty]" overrides (ty = 4 or 8 rows per block), "0": the stage
// passes' geometry.
void energy_geometry(lat_ctx *c)
{
    c->en_pf = c->en_zc = c->en_ty = c->en_nblocks = 0;
    if (!c->rows || c->batch) return;
    int pf = 0, zc = 0, ty = c->rows_ty;
    if (c->N == 256 && c->rows_ty == 4) {
        pf = c->f32 ? 2 : 1;
        zc = 32;
        ty = c->f32 ? 4 : 8;
    }
    if (const char *e = std::getenv("LATTICE_ENERGY_GEOM"))
        if (std::sscanf(e, "%d,%d,%d", &pf, &zc, &ty) < 2) pf = zc = 0;
    if (pf < 1 || pf > 3 || zc < 1 || zc > c->N || (ty != 4 && ty != 8)) return;
    c->en_pf = pf;
    c->en_zc = zc;
    c->en_ty = ty;
    c->en_nblocks = ((c->N + ty - 1) / ty) * ((c->N + zc - 1) / zc);
}

void geometry_from_env(lat_ctx *c)
{
    // prefetch depth of the whole-row kernel at N = 256: two planes in float64
    // (3% faster than one; three spill to 118 AGPRs and ran 5% slower), four in
    // float32 with 4-row blocks and 16-byte accesses (116 against 120 us at two
    // or three); one elsewhere.  LATTICE_ROWS_PF=1..4 overrides (depths above one
    // are instantiated at N = 256 only: two planes for 4-row blocks and for
    // float32 8-row blocks, three for 4-row blocks, four for float32 4-row
    // blocks with 16-byte accesses; other requests fall back to one plane)
    c->rows_pf = c->N == 256 ? (c->f32 ? 4 : 2) : 1;
    if (const char *pf = std::getenv("LATTICE_ROWS_PF")) c->rows_pf = std::min(4, std::max(1, std::atoi(pf)));
    // 16-byte row accesses (four sites per lane) for float32 at N = 256, where
    // they measured 1.2% faster; float64 keeps one site per lane and access
    // (16-byte accesses measured 4% slower at 256^3, as did a 16-byte 4-in-4-out
    // streaming probe against the 8-byte one).  LATTICE_ROWS_VW=1|2|4 overrides
    // where the row holds a whole number of 16-byte vectors per lane.
    const int vmax = c->f32 ? 4 : 2;
    const bool vok = (c->N / 64) % vmax == 0;
    c->rows_vw = (c->f32 && vok) ? vmax : 1;
    if (const char *vw = std::getenv("LATTICE_ROWS_VW")) c->rows_vw = (std::atoi(vw) > 1 && vok) ? vmax : 1;
    // block order at N = 256: y tile fastest (each XCD's blocks form a z slab),
    // measured about 1% faster than y slabs in both precisions; LATTICE_ROWS_YFAST=0|1
    c->rows_y_fastest = c->N == 256 ? 1 : 0;
    if (const char *yo = std::getenv("LATTICE_ROWS_YFAST")) c->rows_y_fastest = std::atoi(yo) != 0;
    // alternating z marches with ordinary stores at N = 256: the next pass
    // starts on the planes still held in the memory-side cache (2% faster in
    // float64, 5% in float32; either change alone measured no gain);
    // LATTICE_ROWS_ALT=0|1 overrides
    c->rows_alternate = c->N == 256 ? 1 : 0;
    if (const char *al = std::getenv("LATTICE_ROWS_ALT")) c->rows_alternate = std::atoi(al) != 0;
    // store policy at N = 256 in float64: non-temporal stores over the first
    // six eighths of the march, ordinary stores over the rest (196.5 against
    // 207.7 us a pass; splits of 2 .. 7 eighths measured 1 .. 5 us slower).
    // LATTICE_ROWS_STORES=0|1 and LATTICE_ROWS_SPLIT=0..8 override
    c->rows_lp = (c->N == 256 && !c->f32) ? 1 : 0;
    if (const char *lp = std::getenv("LATTICE_ROWS_STORES")) c->rows_lp = std::atoi(lp) != 0;
    c->rows_split = 6;
    if (const char *sp = std::getenv("LATTICE_ROWS_SPLIT")) c->rows_split = std::min(8, std::max(0, std::atoi(sp)));
    // opposite marches of neighbouring z chunks (so both read the planes at
    // their common boundary at the same time) at N = 256 in float32: 105.2
    // against 106.2 us; float64 ran slower with it (208 against 195 us, with
    // its store policy).  LATTICE_ROWS_ZPAIR=0|1 overrides
    c->rows_zpair = (c->N == 256 && c->f32) ? 1 : 0;
    if (const char *zp = std::getenv("LATTICE_ROWS_ZPAIR")) c->rows_zpair = std::atoi(zp) != 0;
    const char *s = std::getenv("LATTICE_TILE");
    if (s && std::strncmp(s, "rows", 4) == 0 && rows_ok(c->N)) {
        int ty = 8, z = 0;
        std::sscanf(s + 4, ",%d,%d", &ty, &z);
        if (ty != 4) ty = 8;
        set_rows_geometry(c, ty, z);
        return;
    }
    int tile = pick_tile(c->N), zc = 0;
    if (s) {
        int tx = 0, ty = 0, z = 0;
        if (std::sscanf(s, "%d,%d,%d", &tx, &ty, &z) >= 2) {
            for (int i = 0; i < kNumTiles; ++i)
                if (kTiles[i].tx == tx && kTiles[i].ty == ty) tile = i;
            zc = z;
            set_geometry(c, tile, zc);
            return;
        }
    }
    if (rows_ok(c->N)) {
        // measured on the 256^3 two-field pass: 4-row blocks with loads two
        // planes ahead in both precisions (float32 with 16-byte accesses: 1%
        // faster than 8-row blocks with one plane ahead); 8-row blocks for
        // float32 at N = 64, 128
        set_rows_geometry(c, (c->f32 && c->N != 256) ? 8 : 4, 0);
        return;
    }
    set_geometry(c, tile, zc);
}

// ---------------------------------------------------------------------------
// kernel dispatch
// ---------------------------------------------------------------------------
template <typename T, int NF, int TX, int TY>
hipError_t launch_variant(int variant, const ScalarArgs<T> &a, int nb, hipStream_t s)
{
    const dim3 grid(nb), block(TX * TY);
    switch (variant) {
    case kKickOnly:
        hipLaunchKernelGGL((scalar_stage<T, NF, TX, TY, false, false, false, false, true>), grid, block, 0, s, a);
        break;
    case kKickOnlyRed:
        hipLaunchKernelGGL((scalar_stage<T, NF, TX, TY, false, false, true, false, true>), grid, block, 0, s, a);
        break;
    case kDriftKick:
        hipLaunchKernelGGL((scalar_stage<T, NF, TX, TY, true, false, false, true, true>), grid, block, 0, s, a);
        break;
    case kDriftKickRed:
        hipLaunchKernelGGL((scalar_stage<T, NF, TX, TY, true, false, true, true, true>), grid, block, 0, s, a);
        break;
    case kKickDrift:
        hipLaunchKernelGGL((scalar_stage<T, NF, TX, TY, false, true, false, true, true>), grid, block, 0, s, a);
        break;
    case kEnergy:
        hipLaunchKernelGGL((scalar_stage<T, NF, TX, TY, false, false, true, false, false>), grid, block, 0, s, a);
        break;
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename T, int NF, int XS, int TY, int PF = 1, int VW = 1, int LP = 0>
hipError_t launch_rows_variant(int variant, const ScalarArgs<T> &a, int nb, hipStream_t s)
{
    const dim3 grid(nb), block(64 * TY);
    switch (variant) {
    case kKickOnly:
        hipLaunchKernelGGL((scalar_rows<T, NF, XS, TY, false, false, false, false, true, PF, VW, LP>), grid, block, 0, s, a);
        break;
    case kKickOnlyRed:
        hipLaunchKernelGGL((scalar_rows<T, NF, XS, TY, false, false, true, false, true, PF, VW, LP>), grid, block, 0, s, a);
        break;
    case kDriftKick:
        hipLaunchKernelGGL((scalar_rows<T, NF, XS, TY, true, false, false, true, true, PF, VW, LP>), grid, block, 0, s, a);
        break;
    case kDriftKickRed:
        hipLaunchKernelGGL((scalar_rows<T, NF, XS, TY, true, false, true, true, true, PF, VW, LP>), grid, block, 0, s, a);
        break;
    case kKickDrift:
        hipLaunchKernelGGL((scalar_rows<T, NF, XS, TY, false, true, false, true, true, PF, VW, LP>), grid, block, 0, s, a);
        break;
    case kEnergy:
        hipLaunchKernelGGL((scalar_rows<T, NF, XS, TY, false, false, true, false, false, PF, VW, LP>), grid, block, 0, s, a);
        break;
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// pf: prefetch depth in planes (2 is instantiated for N = 256 with 4-row
// blocks only; 8-row float64 blocks would spill at that depth).
// vw > 1: 16-byte accesses (two float64 or four float32 sites per lane and
// access), instantiated where the row holds a whole number of them per lane:
// N = 128, 256 in float64, N = 256 in float32.
// lp: store policy of the row kernel (RowPolicy in stage_rows.hpp; 1 streams
// the first part of the march past the caches), instantiated for the N = 256
// defaults (float64 4-row blocks two planes ahead, float32 4-row blocks four
// planes ahead with 16-byte accesses); elsewhere policy 0.
template <typename T, int NF>
hipError_t launch_rows(int N, int ty, int pf, int vw, int variant, const ScalarArgs<T> &a, int nb, hipStream_t s,
                       int lp = 0)
{
    const int xs = N / 64;
    constexpr int V = 16 / (int)sizeof(T);
    if constexpr (sizeof(T) == 8) {
        if (lp == 1 && vw == 1 && pf == 2 && xs == 4 && ty == 4)
            return launch_rows_variant<T, NF, 4, 4, 2, 1, 1>(variant, a, nb, s);
    } else {
        if (lp == 1 && vw > 1 && pf == 4 && xs == 4 && ty == 4)
            return launch_rows_variant<T, NF, 4, 4, 4, V, 1>(variant, a, nb, s);
    }
    if (vw > 1 && xs % V == 0) {
        if (pf == 2 && xs == 4 && ty == 4) return launch_rows_variant<T, NF, 4, 4, 2, V>(variant, a, nb, s);
        if constexpr (V == 4) {
            if (pf == 2 && xs == 4 && ty == 8) return launch_rows_variant<T, NF, 4, 8, 2, V>(variant, a, nb, s);
            if (pf == 3 && xs == 4 && ty == 4) return launch_rows_variant<T, NF, 4, 4, 3, V>(variant, a, nb, s);
            if (pf == 4 && xs == 4 && ty == 4) return launch_rows_variant<T, NF, 4, 4, 4, V>(variant, a, nb, s);
        }
        if (xs == 4) return ty == 4 ? launch_rows_variant<T, NF, 4, 4, 1, V>(variant, a, nb, s)
                                    : launch_rows_variant<T, NF, 4, 8, 1, V>(variant, a, nb, s);
        if constexpr (V == 2) {
            if (xs == 2) return ty == 4 ? launch_rows_variant<T, NF, 2, 4, 1, V>(variant, a, nb, s)
                                        : launch_rows_variant<T, NF, 2, 8, 1, V>(variant, a, nb, s);
        }
        return hipErrorInvalidValue;
    }
    if (pf == 2 && xs == 4 && ty == 4) return launch_rows_variant<T, NF, 4, 4, 2>(variant, a, nb, s);
    if constexpr (sizeof(T) == 8) {
        if (pf == 3 && xs == 4 && ty == 4) return launch_rows_variant<T, NF, 4, 4, 3>(variant, a, nb, s);
    }
    if (ty == 4) {
        if (xs == 1) return launch_rows_variant<T, NF, 1, 4>(variant, a, nb, s);
        if (xs == 2) return launch_rows_variant<T, NF, 2, 4>(variant, a, nb, s);
        if (xs == 4) return launch_rows_variant<T, NF, 4, 4>(variant, a, nb, s);
    } else {
        if (xs == 1) return launch_rows_variant<T, NF, 1, 8>(variant, a, nb, s);
        if (xs == 2) return launch_rows_variant<T, NF, 2, 8>(variant, a, nb, s);
        if (xs == 4) return launch_rows_variant<T, NF, 4, 8>(variant, a, nb, s);
    }
    return hipErrorInvalidValue;
}

template <typename T, int NF>
hipError_t launch_tile(int tile, int variant, const ScalarArgs<T> &a, int nb, hipStream_t s)
{
    switch (tile) {
    case 0: return launch_variant<T, NF, 64, 4>(variant, a, nb, s);
    case 1: return launch_variant<T, NF, 64, 8>(variant, a, nb, s);
    case 2: return launch_variant<T, NF, 32, 8>(variant, a, nb, s);
    case 3: return launch_variant<T, NF, 16, 16>(variant, a, nb, s);
    case 4: return launch_variant<T, NF, 8, 8>(variant, a, nb, s);
    }
    return hipErrorInvalidValue;
}

// Which arrays a variant reads with a halo (must not be written in place) and writes.
struct VariantIO {
    bool wphi, wpi, pi_halo;
};
VariantIO variant_io(int v)
{
    switch (v) {
    case kKickOnly:
    case kKickOnlyRed: return {false, true, false};
    case kDriftKick:
    case kDriftKickRed: return {true, true, true};
    case kKickDrift: return {true, true, false};
    default: return {false, false, false};
    }
}

// ---------------------------------------------------------------------------
// event timing of launches (profiling mode)
// ---------------------------------------------------------------------------
lat_status get_event(lat_ctx *c, hipEvent_t *ev)
{
    if (!c->spare.empty()) {
        *ev = c->spare.back();
        c->spare.pop_back();
        return LAT_OK;
    }
    HIPCHK(c, hipEventCreate(ev));
    return LAT_OK;
}

lat_status timing_begin(lat_ctx *c, hipEvent_t *e0, hipEvent_t *e1)
{
    lat_status s;
    if ((s = get_event(c, e0)) != LAT_OK) return s;
    if ((s = get_event(c, e1)) != LAT_OK) return s;
    HIPCHK(c, hipEventRecord(*e0, c->stream));
    return LAT_OK;
}

lat_status timing_end(lat_ctx *c, hipEvent_t e0, hipEvent_t e1, int kind)
{
    HIPCHK(c, hipEventRecord(e1, c->stream));
    c->timed.push_back({e0, e1, kind});
    return LAT_OK;
}

lat_status harvest_timing(lat_ctx *c)
{
    for (auto &t : c->timed) {
        HIPCHK(c, hipEventSynchronize(t.stop));
        float ms = 0.0f;
        HIPCHK(c, hipEventElapsedTime(&ms, t.start, t.stop));
        c->kernel_ms[t.kind] += ms;
        c->spare.push_back(t.start);
        c->spare.push_back(t.stop);
    }
    c->timed.clear();
    return LAT_OK;
}

// Deferred finalisation of a pass (see ScalarArgs): where its block sums go
// and which earlier sums its prologue finalises.
struct PassLink {
    int defer = 0;
    double *partials = nullptr;    // this pass's block sums (defer = 1)
    const double *fin = nullptr;   // previous pass's block sums to finalise, or null
    int fin_mode = kLastSelf;
    const PassCoef *fin_coef = nullptr;
    const ScaleRecord *fin_in = nullptr;
    ScaleRecord *fin_out = nullptr;
    // defer = 1 on a store-only pass: sums_finish adds this pass's block sums
    // into store_to->sums right after it (inside the pass's timed region)
    ScaleRecord *store_to = nullptr;
};

// The deferred block sums of a store-only pass (the energy pass), added by one
// block of NT threads (NT as the pass's, so in the order of the last-block
// reduction) into Sout->sums: the same values as that reduction, with no
// ticket release in the pass's blocks.
template <int NT, int NQ>
__global__ void __launch_bounds__(NT) sums_finish(const double *partials, int nb, ScaleRecord *Sout)
{
    __shared__ double lds_red[(NT / 64) * NQ];
    const int tid = threadIdx.x;
    double part[NQ];
#pragma unroll
    for (int k = 0; k < NQ; ++k) part[k] = 0.0;
    for (int i = tid; i < nb; i += NT) {
#pragma unroll
        for (int k = 0; k < NQ; ++k) part[k] += partials[(size_t)i * NQ + k];
    }
    double fin[NQ];
    block_sums<NT, NQ>(part, lds_red, fin);
    if (tid == 0) {
#pragma unroll
        for (int k = 0; k < NQ; ++k) Sout->sums[k] = fin[k];
    }
}

hipError_t launch_sums_finish(int NT, int nf, const double *partials, int nb, ScaleRecord *S, hipStream_t st)
{
#define SUMS_FIN(nt)                                                                                       \
    if (NT == nt) {                                                                                        \
        if (nf == 1) hipLaunchKernelGGL((sums_finish<nt, 3>), dim3(1), dim3(nt), 0, st, partials, nb, S); \
        else hipLaunchKernelGGL((sums_finish<nt, 6>), dim3(1), dim3(nt), 0, st, partials, nb, S);         \
        return hipGetLastError();                                                                          \
    }
    SUMS_FIN(64)
    SUMS_FIN(128)
    SUMS_FIN(256)
    SUMS_FIN(512)
#undef SUMS_FIN
    return hipErrorInvalidValue;
}

// The deferred block partials of a gauge summing pass (the U(1) and SU(2)
// energy and kick-and-sums passes: 8 sums, then 3 maxima per block), combined
// by one block of NT threads, NT the pass's block size: the order and the
// arithmetic of the pass's own last-block reduction.
static_assert(kU1Sums == 8 && kU1Maxes == 3 && kSU2Sums == 8 && kSU2Maxes == 3, "gauge sum layout");
template <int NT>
__global__ void __launch_bounds__(NT) gauge_sums_finish(const double *partials, int nb, ScaleRecord *S)
{
    constexpr int NS = 8, NQ = 11;
    __shared__ double lds_red[(NT / 64) * NQ];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    double part[NQ];
#pragma unroll
    for (int k = 0; k < NQ; ++k) part[k] = 0.0;
    for (int i = tid; i < nb; i += NT) {
#pragma unroll
        for (int k = 0; k < NQ; ++k) {
            const double v = partials[(size_t)i * NQ + k];
            part[k] = k < NS ? part[k] + v : fmax(part[k], v);
        }
    }
#pragma unroll
    for (int k = 0; k < NQ; ++k) {
        const double r = k < NS ? wave_sum(part[k]) : wave_max(part[k]);
        if (lane == 0) lds_red[w * NQ + k] = r;
    }
    __syncthreads();
    if (tid == 0) {
        for (int k = 0; k < NQ; ++k) {
            double r = 0.0;
            for (int i = 0; i < NT / 64; ++i) r = k < NS ? r + lds_red[i * NQ + k] : fmax(r, lds_red[i * NQ + k]);
            if (k < NS) S->sums[k] = r;
            else S->maxes[k - NS] = r;
        }
    }
}

hipError_t launch_gauge_sums_finish(int NT, const double *partials, int nb, ScaleRecord *S, hipStream_t st)
{
    if (NT == 256) hipLaunchKernelGGL(gauge_sums_finish<256>, dim3(1), dim3(256), 0, st, partials, nb, S);
    else if (NT == 512) hipLaunchKernelGGL(gauge_sums_finish<512>, dim3(1), dim3(512), 0, st, partials, nb, S);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

// Summing passes of the gauge models leave their block partials to
// gauge_sums_finish (no ticket release in their blocks); LATTICE_ENERGY_DEFER=0
// keeps the ticketed last block (the same results, bit for bit).
static bool gauge_defer_on()
{
    const char *e = std::getenv("LATTICE_ENERGY_DEFER");
    return e ? std::atoi(e) != 0 : true;
}

template <typename T>
lat_status run_pass_t(lat_ctx *c, int variant, int pass_index, int last_mode, hipStream_t stream,
                      const PassLink *lk = nullptr)
{
    const VariantIO io = variant_io(variant);
    ScalarArgs<T> a{};
    for (int f = 0; f < c->nf; ++f) {
        const int cp = c->cur_phi[f], cq = c->cur_pi[f];
        a.phi_in[f] = (const T *)c->phi[f][cp];
        a.pi_in[f] = (const T *)c->pi[f][cq];
        a.phi_out[f] = io.wphi ? (T *)c->phi[f][cp ^ 1] : nullptr;
        a.pi_out[f] = io.wpi ? (io.pi_halo ? (T *)c->pi[f][cq ^ 1] : (T *)c->pi[f][cq]) : nullptr;
    }
    a.N = c->N;
    a.zc = c->zc;
    a.tiles_x = c->tiles_x;
    a.tiles_y = c->tiles_y;
    a.y_fastest = c->rows_y_fastest;
    // whole-row kernel: odd passes of a call march down, so each pass starts on
    // the planes the pass before it wrote last (fixed by the pass's place in the
    // call, so graph replays and direct launches take the same directions), and
    // outputs go through the caches so that those planes are still there
    a.down = c->rows_alternate ? (pass_index & 1) : 0;
    a.zpair = c->rows_zpair;
    a.cached_out = c->rows_alternate;
    a.split = c->rows_split;
    a.inv_dx2 = 1.0 / (c->p.dx * c->p.dx);
    a.lam = c->p.lambda;
    a.q = c->p.potential == LAT_PHI4_CHI2 ? c->p.q : 0.0;
    a.coef = c->coef + pass_index;
    a.coef_next = c->coef + pass_index + 1;
    a.partials = c->partials;
    a.ticket = c->ticket;
    a.sc = c->sc;
    a.last_mode = last_mode;
    a.alpha = c->p.alpha;
    a.kappa2 = c->p.kappa2;
    a.inv_vol = 1.0 / (double)c->vol;
    if (lk) {
        a.defer = lk->defer;
        if (lk->defer) a.partials = lk->partials;
        a.fin = lk->fin;
        a.fin_nb = c->nblocks;
        a.fin_mode = lk->fin_mode;
        a.fin_coef = lk->fin_coef;
        a.fin_in = lk->fin_in;
        a.fin_out = lk->fin_out;
    }
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    if (c->profiling) {
        lat_status st = timing_begin(c, &ev0, &ev1);
        if (st != LAT_OK) return st;
    }
    hipError_t e;
    int nb = c->nblocks, pf = c->rows_pf, lp = c->rows_lp, ty = c->rows_ty;
    if (variant == kEnergy && c->rows && c->en_nblocks > 0) {
        a.zc = c->en_zc;
        ty = c->en_ty;
        a.tiles_y = (c->N + ty - 1) / ty;
        nb = c->en_nblocks;
        pf = c->en_pf;
        lp = 0;
    }
    if (c->rows)
        e = c->nf == 1 ? launch_rows<T, 1>(c->N, ty, pf, c->rows_vw, variant, a, nb, stream, lp)
                       : launch_rows<T, 2>(c->N, ty, pf, c->rows_vw, variant, a, nb, stream, lp);
    else
        e = c->nf == 1 ? launch_tile<T, 1>(c->tile, variant, a, c->nblocks, stream)
                       : launch_tile<T, 2>(c->tile, variant, a, c->nblocks, stream);
    if (e != hipSuccess) return fail(c, LAT_EHIP, std::string("stage launch: ") + hipGetErrorString(e));
    if (lk && lk->defer && lk->store_to) {
        const int NT = c->rows ? 64 * ty : kTiles[c->tile].tx * kTiles[c->tile].ty;
        e = launch_sums_finish(NT, c->nf, lk->partials, c->rows ? nb : c->nblocks, lk->store_to, stream);
        if (e != hipSuccess) return fail(c, LAT_EHIP, std::string("sums launch: ") + hipGetErrorString(e));
    }
    if (c->profiling) {
        lat_status st = timing_end(c, ev0, ev1, variant);
        if (st != LAT_OK) return st;
    }
    c->launches[variant] += 1;
    for (int f = 0; f < c->nf; ++f) {
        if (io.wphi) c->cur_phi[f] ^= 1;
        if (io.wpi && io.pi_halo) c->cur_pi[f] ^= 1;
    }
    return LAT_OK;
}

lat_status run_pass(lat_ctx *c, int variant, int pass_index, int last_mode, hipStream_t stream,
                    const PassLink *lk = nullptr)
{
    return c->f32 ? run_pass_t<float>(c, variant, pass_index, last_mode, stream, lk)
                  : run_pass_t<double>(c, variant, pass_index, last_mode, stream, lk);
}

// the deferred-finalisation chain of a call's passes 0 .. M (all reducing and
// deferring except where the caller says): pass p >= 1 finalises pass p - 1
// from the record R_{p-2} (the context's record for p = 1) into R_{p-1}; the
// two block-sum buffers and the two spare records alternate by pass parity
PassLink pass_link(lat_ctx *c, int64_t p, int mode, bool defer)
{
    PassLink lk;
    double *buf[2] = {c->partials, c->partials + (size_t)c->nblocks * 8};
    ScaleRecord *tmp[2] = {c->sc + 1, c->sc + 2};
    lk.defer = defer ? 1 : 0;
    lk.partials = buf[p & 1];
    if (p >= 1) {
        lk.fin = buf[(p - 1) & 1];
        lk.fin_mode = mode;
        lk.fin_coef = c->coef + (p - 1);
        lk.fin_in = p == 1 ? c->sc : tmp[(p - 2) & 1];
        lk.fin_out = tmp[(p - 1) & 1];
    }
    return lk;
}

// the finaliser after the last deferring pass M of a call: its sums, applied
// to R_{M-1}, give the context's record
lat_status finish_chain(lat_ctx *c, int64_t M, int mode, hipStream_t st)
{
    double *buf[2] = {c->partials, c->partials + (size_t)c->nblocks * 8};
    const ScaleRecord *in = M == 0 ? c->sc : c->sc + 1 + ((M - 1) & 1);
    const double iv = 1.0 / (double)c->vol, idx2 = 1.0 / (c->p.dx * c->p.dx);
    const int NT = c->rows ? 64 * c->rows_ty : kTiles[c->tile].tx * kTiles[c->tile].ty;
    const double *P = buf[M & 1];
    PassCoef *Nx = c->coef + M + 1;
    if (NT == 64) {
        if (c->nf == 1)
            hipLaunchKernelGGL((self_finish<64, 1>), dim3(1), dim3(64), 0, st, P, c->nblocks, mode, c->coef + M, in,
                               c->sc, Nx, c->p.alpha, c->p.kappa2, iv, idx2);
        else
            hipLaunchKernelGGL((self_finish<64, 2>), dim3(1), dim3(64), 0, st, P, c->nblocks, mode, c->coef + M, in,
                               c->sc, Nx, c->p.alpha, c->p.kappa2, iv, idx2);
    } else if (NT == 256) {
        if (c->nf == 1)
            hipLaunchKernelGGL((self_finish<256, 1>), dim3(1), dim3(256), 0, st, P, c->nblocks, mode, c->coef + M, in,
                               c->sc, Nx, c->p.alpha, c->p.kappa2, iv, idx2);
        else
            hipLaunchKernelGGL((self_finish<256, 2>), dim3(1), dim3(256), 0, st, P, c->nblocks, mode, c->coef + M, in,
                               c->sc, Nx, c->p.alpha, c->p.kappa2, iv, idx2);
    } else if (NT == 512) {
        if (c->nf == 1)
            hipLaunchKernelGGL((self_finish<512, 1>), dim3(1), dim3(512), 0, st, P, c->nblocks, mode, c->coef + M, in,
                               c->sc, Nx, c->p.alpha, c->p.kappa2, iv, idx2);
        else
            hipLaunchKernelGGL((self_finish<512, 2>), dim3(1), dim3(512), 0, st, P, c->nblocks, mode, c->coef + M, in,
                               c->sc, Nx, c->p.alpha, c->p.kappa2, iv, idx2);
    } else {
        return fail(c, LAT_EHIP, "unexpected block size for the finaliser");
    }
    HIPCHK(c, hipGetLastError());
    return LAT_OK;
}

lat_status run_pass(lat_ctx *c, int variant, int pass_index, int last_mode)
{
    return run_pass(c, variant, pass_index, last_mode, c->stream);
}

// Enqueue the pass launches of one lattice_step call.  Outside profiling,
// calls of at least kGraphMinPasses passes are captured once into a HIP graph
// per (step count, leapfrog phase) and replayed; shorter calls launch directly,
// where a graph launch costs more than it saves.  The per-call coefficient
// table is uploaded before, outside the graph, so a replay reads the current
// coefficients.  Buffer bookkeeping at the start of a call is always the
// caller's arrays (settled), so a replay ends in the same buffer state as the
// captured launches.
constexpr int64_t kGraphMinPasses = 8;
// longest run of stencil passes one lattice_step call enqueues as a unit
// (longer calls are split into chunks of this size)
constexpr int64_t kChunkPasses = 1024;

void drop_step_graphs(lat_ctx *c)
{
    for (auto &g : c->sg) {
        if (g.exec) (void)hipGraphExecDestroy(g.exec);
        g = lat_ctx::StepGraph{};
    }
}

template <typename F>
lat_status launch_passes(lat_ctx *c, int64_t key_n, int64_t passes, F &&enqueue)
{
    if (c->profiling || passes < kGraphMinPasses || std::getenv("LATTICE_NO_GRAPH")) return enqueue(c->stream);
    for (int f = 0; f < c->nf; ++f)
        if (c->cur_phi[f] || c->cur_pi[f]) return enqueue(c->stream);
    if (!c->capture_stream && hipStreamCreateWithFlags(&c->capture_stream, hipStreamNonBlocking) != hipSuccess)
        return enqueue(c->stream);
    lat_ctx::StepGraph *hit = nullptr, *victim = &c->sg[0];
    for (auto &g : c->sg) {
        if (g.exec && g.n == key_n && g.stag == c->lf_stag) hit = &g;
        if (!g.exec || (victim->exec && g.used < victim->used)) victim = &g;
    }
    if (!hit) {
        lat_ctx::StepGraph &g = *victim;
        if (g.exec) HIPCHK(c, hipGraphExecDestroy(g.exec));
        g = lat_ctx::StepGraph{};
        const int stag0 = c->lf_stag;
        int64_t before[8];
        std::memcpy(before, c->launches, sizeof(before));
        HIPCHK(c, hipStreamBeginCapture(c->capture_stream, hipStreamCaptureModeThreadLocal));
        lat_status st = enqueue(c->capture_stream);
        hipGraph_t graph = nullptr;
        hipError_t e = hipStreamEndCapture(c->capture_stream, &graph);
        if (st != LAT_OK) {
            if (graph) (void)hipGraphDestroy(graph);
            return st;
        }
        if (e != hipSuccess) return fail(c, LAT_EHIP, std::string("graph capture: ") + hipGetErrorString(e));
        e = hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e != hipSuccess) {
            g.exec = nullptr;
            return fail(c, LAT_EHIP, std::string("graph instantiate: ") + hipGetErrorString(e));
        }
        for (int i = 0; i < 8; ++i) g.launches[i] = c->launches[i] - before[i];
        for (int f = 0; f < 2; ++f) {
            g.end_phi[f] = c->cur_phi[f];
            g.end_pi[f] = c->cur_pi[f];
        }
        g.n = key_n;
        g.stag = stag0;
        hit = &g;
    } else {
        for (int i = 0; i < 8; ++i) c->launches[i] += hit->launches[i];
        for (int f = 0; f < 2; ++f) {
            c->cur_phi[f] = hit->end_phi[f];
            c->cur_pi[f] = hit->end_pi[f];
        }
    }
    hit->used = ++c->sg_clock;
    HIPCHK(c, hipGraphLaunch(hit->exec, c->stream));
    return LAT_OK;
}

// ---------------------------------------------------------------------------
// coefficient tables
// ---------------------------------------------------------------------------
// Coefficient tables start with room for 2048 kick points (192 KB on the
// device, four pinned staging slots of the same size) and at least double
// when a call needs more, so that calls after the first rarely allocate (the
// growth frees and reallocates, which synchronises and drops captured graphs).
constexpr size_t kCoefInitial = 2048;

lat_status reserve_coef(lat_ctx *c, size_t n)
{
    if (n > c->coef_cap) {
        // captured graphs hold the table's address: drop them with it
        drop_step_graphs(c);
        c->graph_n = 0;
        if (c->coef) HIPCHK(c, hipFree(c->coef));
        c->coef = nullptr;
        const size_t cap = std::max(n, std::max(kCoefInitial, 2 * c->coef_cap));
        if (hipMalloc(&c->coef, cap * sizeof(PassCoef)) != hipSuccess)
            return fail(c, LAT_ENOMEM, "coefficient table allocation failed");
        c->coef_cap = cap;
    }
    if (n > c->ring_cap) {
        for (int i = 0; i < lat_ctx::kRing; ++i) {
            if (c->ring_pending[i]) HIPCHK(c, hipEventSynchronize(c->ring_ev[i]));
            c->ring_pending[i] = false;
        }
        if (c->ring_base) HIPCHK(c, hipHostFree(c->ring_base));
        c->ring_base = nullptr;
        const size_t cap = std::max(n, std::max(kCoefInitial, 2 * c->ring_cap));
        if (hipHostMalloc((void **)&c->ring_base, lat_ctx::kRing * cap * sizeof(PassCoef), hipHostMallocDefault) !=
            hipSuccess)
            return fail(c, LAT_ENOMEM, "pinned coefficient staging allocation failed");
        c->ring_cap = cap;
    }
    c->ring_slot = (c->ring_slot + 1) % lat_ctx::kRing;
    const int k = c->ring_slot;
    if (c->ring_pending[k]) {
        HIPCHK(c, hipEventSynchronize(c->ring_ev[k]));
        c->ring_pending[k] = false;
    }
    c->coef_host = c->ring_base + (size_t)k * c->ring_cap;
    std::memset(c->coef_host, 0, n * sizeof(PassCoef));
    return LAT_OK;
}

lat_status upload_coef(lat_ctx *c, size_t n)
{
    const int k = c->ring_slot;
    if (!c->traj_rec)
        for (size_t i = 0; i < n; ++i) c->coef_host[i].traj = nullptr;
    HIPCHK(c, hipMemcpyAsync(c->coef, c->coef_host, n * sizeof(PassCoef), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipEventRecord(c->ring_ev[k], c->stream));
    c->ring_pending[k] = true;
    return LAT_OK;
}

// copy shadow buffers back so the caller's arrays hold the state
lat_status settle(lat_ctx *c)
{
    const size_t bytes = c->vol * c->esize;
    for (int f = 0; f < c->nf; ++f) {
        if (c->cur_phi[f]) {
            HIPCHK(c, hipMemcpyAsync(c->phi[f][0], c->phi[f][1], bytes, hipMemcpyDeviceToDevice, c->stream));
            c->cur_phi[f] = 0;
        }
        if (c->cur_pi[f]) {
            HIPCHK(c, hipMemcpyAsync(c->pi[f][0], c->pi[f][1], bytes, hipMemcpyDeviceToDevice, c->stream));
            c->cur_pi[f] = 0;
        }
    }
    for (int i = 0; i < 3; ++i) {
        if (c->cur_A[i]) {
            HIPCHK(c, hipMemcpyAsync(c->A[i][0], c->A[i][1], bytes, hipMemcpyDeviceToDevice, c->stream));
            c->cur_A[i] = 0;
        }
    }
    if (c->cur_su2) {
        for (int k = 0; k < 4; ++k)
            HIPCHK(c, hipMemcpyAsync(c->dbl[k][0], c->dbl[k][1], bytes, hipMemcpyDeviceToDevice, c->stream));
        for (int k = 0; k < 12; ++k)
            HIPCHK(c, hipMemcpyAsync(c->lnk[k][0], c->lnk[k][1], bytes, hipMemcpyDeviceToDevice, c->stream));
        c->cur_su2 = 0;
    }
    return LAT_OK;
}

// ---------------------------------------------------------------------------
// scalar schedules
// ---------------------------------------------------------------------------
// Leapfrog with self-consistent expansion (reading A3): the drift after each
// kick needs b after that kick, which needs the kicked momenta's volume sum, so
// the drift moves into the next pass (drift on load) and the call ends with a
// drift-only pass.  Pass k < ns kicks pi by c1 (h/2 for the first kick from
// synchronised momenta, else h) and reduces the kicked momenta squared, E_G and
// E_V; its last block kicks b and drifts a (self_update_lf) and writes the next
// pass's drift and kick factors.  Pass ns drifts phi only.
lat_status step_lf_self(lat_ctx *c, int64_t ns, int dir)
{
    const double h = dir * c->p.dt;
    const double al = c->p.alpha;
    lat_status s = reserve_coef(c, (size_t)ns + 2);
    if (s != LAT_OK) return s;
    const double t_start = c->t;
    int stag = c->lf_stag;
    for (int64_t k = 0; k <= ns; ++k) {
        PassCoef &P = c->coef_host[k];
        P.t = t_start + (double)k * h;
        if (k == ns) {   // drift only
            P.c1 = P.c2 = 0.0;
            P.t_next = P.t;
            continue;
        }
        P.c1 = (stag == 0) ? 0.5 * h : h;
        P.c2 = 0.0;
        P.cL = (stag == 0) ? 0.0 : 0.5 * h;
        P.cR = 0.5 * h;
        P.h = h;
        P.t_next = P.t + h;
        stag = dir;
    }
    if ((s = upload_coef(c, (size_t)ns + 2)) != LAT_OK) return s;
    s = launch_passes(c, dir * ns, ns + 1, [&](hipStream_t st) {
        hipLaunchKernelGGL(self_prologue, dim3(1), dim3(64), 0, st, c->coef, c->sc, al);
        HIPCHK(c, hipGetLastError());
        for (int64_t k = 0; k <= ns; ++k) {
            const int v = k == ns ? kDriftKick : (k == 0 ? kKickOnlyRed : kDriftKickRed);
            // the drift-only pass finalises the last kick's sums and reduces nothing
            const PassLink lk = pass_link(c, k, kLastSelfLF, k < ns);
            lat_status r = run_pass(c, v, (int)k, k == ns ? kLastStore : kLastSelfLF, st, &lk);
            if (r != LAT_OK) return r;
        }
        // the record the drift-only pass wrote is the context's
        hipLaunchKernelGGL(record_copy, dim3(1), dim3(64), 0, st, (const ScaleRecord *)(c->sc + 1 + ((ns - 1) & 1)),
                           c->sc);
        HIPCHK(c, hipGetLastError());
        return LAT_OK;
    });
    if (s != LAT_OK) return s;
    c->lf_stag = dir;
    c->t = t_start + (double)ns * h;
    return LAT_OK;
}

// Temporal blocking for small lattices (stage_slab.hpp): S leapfrog steps per
// launch, blocks of ZS planes by YB rows, for real scalar lattices with
// N <= 32, S = 2 .. 5 and ZS = 1 or 2 compiled.  The window (ZS + 2 S planes
// by YB + 2 S rows) must not wrap onto itself, its rows of N sites must fit a
// block and its advanced planes the LDS a block may use.  Default S = 4,
// ZS = 1, YB = 4 (at 32^3: 256 blocks of 12 x 32 threads); LATTICE_SLAB=
// "S,ZS[,YB]" overrides, "0" turns it off.
template <typename T, int NF, int S, int ZS>
void slab_kernel_of(const void **fn, size_t *lds, int N, int yb)
{
    *fn = (const void *)lf_slab<T, NF, S, ZS>;
    *lds = slab_lds<T, NF, S, ZS>(N, yb);
}

template <typename T, int NF, int S>
bool slab_pick_zs(int zs, const void **fn, size_t *lds, int N, int yb)
{
    switch (zs) {
    case 1: slab_kernel_of<T, NF, S, 1>(fn, lds, N, yb); return true;
    case 2: slab_kernel_of<T, NF, S, 2>(fn, lds, N, yb); return true;
    default: return false;
    }
}

template <typename T, int NF>
bool slab_pick(int S, int zs, const void **fn, size_t *lds, int N, int yb)
{
    switch (S) {
    case 2: return slab_pick_zs<T, NF, 2>(zs, fn, lds, N, yb);
    case 3: return slab_pick_zs<T, NF, 3>(zs, fn, lds, N, yb);
    case 4: return slab_pick_zs<T, NF, 4>(zs, fn, lds, N, yb);
    case 5: return slab_pick_zs<T, NF, 5>(zs, fn, lds, N, yb);
    default: return false;
    }
}

bool slab_kernel(const lat_ctx *c, int S, int zs, int yb, const void **fn, size_t *lds)
{
    if (c->f32)
        return c->nf == 1 ? slab_pick<float, 1>(S, zs, fn, lds, c->N, yb) : slab_pick<float, 2>(S, zs, fn, lds, c->N, yb);
    return c->nf == 1 ? slab_pick<double, 1>(S, zs, fn, lds, c->N, yb) : slab_pick<double, 2>(S, zs, fn, lds, c->N, yb);
}

void slab_config(lat_ctx *c)
{
    c->slab_steps = c->slab_zs = c->slab_yb = 0;
    c->slab_fn = nullptr;
    c->slab_lds = 0;
    if (c->batch || c->u1 || c->su2 || c->N > 32) return;
    int S = 4, zs = 1, yb = 4;
    if (const char *e = std::getenv("LATTICE_SLAB")) {
        if (std::atoi(e) == 0) return;
        if (std::sscanf(e, "%d,%d,%d", &S, &zs, &yb) < 2) return;
    }
    int lim = 0;
    if (hipDeviceGetAttribute(&lim, hipDeviceAttributeMaxSharedMemoryPerBlock, c->device) != hipSuccess || lim <= 0)
        return;
    const void *fn = nullptr;
    size_t lds = 0;
    // fall back to fewer steps per launch, then fewer rows per block, while
    // the window does not fit
    const int N = c->N;
    for (S = std::min(S, 5); S >= 2; --S) {
        int b = std::min(yb, N - 2 * S);
        while (b >= 1 && (b + 2 * S) * N > kSlabMaxThreads) --b;
        if (b >= 1 && zs + 2 * S <= N && slab_kernel(c, S, zs, b, &fn, &lds) && lds <= (size_t)lim) {
            yb = b;
            break;
        }
    }
    if (S < 2) return;
    if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess) {
        (void)hipGetLastError();
        return;
    }
    c->slab_steps = S;
    c->slab_zs = zs;
    c->slab_yb = yb;
    c->slab_fn = fn;
    c->slab_lds = lds;
}

// one launch of `steps` (1 .. S) leapfrog steps from the coefficients of step `first`
template <typename T>
lat_status slab_launch_t(lat_ctx *c, int64_t first, int steps, hipStream_t st)
{
    SlabArgs<T> a{};
    for (int f = 0; f < c->nf; ++f) {
        a.phi_in[f] = (const T *)c->phi[f][c->cur_phi[f]];
        a.pi_in[f] = (const T *)c->pi[f][c->cur_pi[f]];
        a.phi_out[f] = (T *)c->phi[f][c->cur_phi[f] ^ 1];
        a.pi_out[f] = (T *)c->pi[f][c->cur_pi[f] ^ 1];
    }
    a.N = c->N;
    a.yb = c->slab_yb;
    a.steps = steps;
    a.inv_dx2 = 1.0 / (c->p.dx * c->p.dx);
    a.lam = c->p.lambda;
    a.q = c->p.potential == LAT_PHI4_CHI2 ? c->p.q : 0.0;
    a.coef = c->coef + first;
    const dim3 grid((unsigned)((c->N + c->slab_zs - 1) / c->slab_zs),
                    (unsigned)((c->N + c->slab_yb - 1) / c->slab_yb));
    const dim3 blk((unsigned)((((c->slab_yb + 2 * c->slab_steps) * c->N + 63) / 64) * 64));
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    if (c->profiling) {
        lat_status s = timing_begin(c, &ev0, &ev1);
        if (s != LAT_OK) return s;
    }
    void *args[] = {&a};
    HIPCHK(c, hipLaunchKernel(c->slab_fn, grid, blk, args, c->slab_lds, st));
    if (c->profiling) {
        lat_status s = timing_end(c, ev0, ev1, kKickDrift);
        if (s != LAT_OK) return s;
    }
    c->launches[kKickDrift] += 1;
    for (int f = 0; f < c->nf; ++f) {
        c->cur_phi[f] ^= 1;
        c->cur_pi[f] ^= 1;
    }
    return LAT_OK;
}

lat_status step_lf(lat_ctx *c, int64_t ns, int dir)
{
    if (c->p.expansion == LAT_EXP_SELF) return step_lf_self(c, ns, dir);
    const double h = dir * c->p.dt;
    const double al = c->p.alpha;
    lat_status s = reserve_coef(c, (size_t)ns + 1);
    if (s != LAT_OK) return s;
    const double t_start = c->t;
    int stag = c->lf_stag;
    for (int64_t k = 0; k < ns; ++k) {
        PassCoef &P = c->coef_host[k];
        const double t = t_start + (double)k * h;
        const double a = scale_at(c, t);
        P.ka1 = std::pow(a, 1.0 + al);
        P.ka3 = std::pow(a, 3.0 + al);
        P.c1 = (stag == 0) ? 0.5 * h : h;
        P.c2 = 0.0;
        P.dend = h * std::pow(scale_at(c, t + 0.5 * h), al - 3.0);
        P.t = t;
        stag = dir;
    }
    if ((s = upload_coef(c, (size_t)ns)) != LAT_OK) return s;
    if (c->slab_steps > 0) {
        const int64_t S = c->slab_steps, nl = (ns + S - 1) / S;
        s = launch_passes(c, dir * ns, nl, [&](hipStream_t st) {
            for (int64_t j = 0; j < nl; ++j) {
                const int steps = (int)std::min<int64_t>(S, ns - j * S);
                lat_status r = c->f32 ? slab_launch_t<float>(c, j * S, steps, st)
                                      : slab_launch_t<double>(c, j * S, steps, st);
                if (r != LAT_OK) return r;
            }
            return LAT_OK;
        });
    } else {
        s = launch_passes(c, dir * ns, ns, [&](hipStream_t st) {
            for (int64_t k = 0; k < ns; ++k) {
                lat_status r = run_pass(c, kKickDrift, (int)k, kLastStore, st);
                if (r != LAT_OK) return r;
            }
            return LAT_OK;
        });
    }
    if (s != LAT_OK) return s;
    c->lf_stag = dir;
    c->t = t_start + (double)ns * h;
    return LAT_OK;
}

// Sub-step weights (in units of h) of one velocity-Verlet step of the
// context's order, as symmetric products of VV2 maps (sec. 4.3 VV family):
//   VV2   {1}
//   VV4   triple jump S(x1 h) S(x0 h) S(x1 h), x1 = 1/(2 - 2^{1/3}), x0 = 1 - 2 x1
//   VV6   Yoshida (1990) solution A, 7 maps: y3 y2 y1 y0 y1 y2 y3
//   VV8   Yoshida (1990) solution D, 15 maps: y7 ... y1 y0 y1 ... y7
//   VV10  triple jump of VV8 with c = 2^{1/9}: 45 maps
// where y0 = 1 - 2 (y1 + ... + ym) makes the weights sum to one.
std::vector<double> vv_weights(int integrator)
{
    static const double solA[3] = {-1.17767998417887, 0.235573213359357, 0.784513610477560};
    static const double solD[7] = {0.102799849391985, -1.96061023297549, 1.93813913762276,
                                   -0.158240635368243, -1.44485223686048, 0.253693336566229,
                                   0.914844246229740};
    auto jump = [](const std::vector<double> &inner, double cc) {
        const double x1 = 1.0 / (2.0 - cc), x0 = -cc / (2.0 - cc);
        std::vector<double> out;
        out.reserve(3 * inner.size());
        for (double x : {x1, x0, x1})
            for (double v : inner) out.push_back(x * v);
        return out;
    };
    auto palindrome = [](const double *y, int m) {
        double tot = 0.0;
        for (int i = 0; i < m; ++i) tot += y[i];
        std::vector<double> out;
        out.reserve(2 * m + 1);
        for (int i = m - 1; i >= 0; --i) out.push_back(y[i]);
        out.push_back(1.0 - 2.0 * tot);
        for (int i = 0; i < m; ++i) out.push_back(y[i]);
        return out;
    };
    switch (integrator) {
    case LAT_VV4: return jump({1.0}, std::cbrt(2.0));
    case LAT_VV6: return palindrome(solA, 3);
    case LAT_VV8: return palindrome(solD, 7);
    case LAT_VV10: return jump(palindrome(solD, 7), std::pow(2.0, 1.0 / 9.0));
    default: return {1.0};
    }
}

lat_status step_vv(lat_ctx *c, int64_t ns, int dir)
{
    const double h = dir * c->p.dt;
    const double al = c->p.alpha;
    const bool self = c->p.expansion == LAT_EXP_SELF;
    const std::vector<double> w = vv_weights(c->p.integrator);
    const int J = (int)w.size();
    const int64_t M = (int64_t)J * ns;
    lat_status s = reserve_coef(c, (size_t)M + 2);
    if (s != LAT_OK) return s;
    const double t_start = c->t;
    // sub-step sizes and kick-point times (within a step, accumulated in order)
    auto hs = [&](int64_t p) { return w[p % J] * h; };
    std::vector<double> tp((size_t)M + 1);
    for (int64_t p = 0; p <= M; ++p) {
        if (p == M) tp[p] = t_start + (double)ns * h;
        else if (p % J == 0) tp[p] = t_start + (double)(p / J) * h;
        else tp[p] = tp[p - 1] + hs(p - 1);
    }
    auto ts = [&](int64_t p) { return tp[(size_t)(p < M ? p : M)]; };
    for (int64_t p = 0; p <= M; ++p) {
        PassCoef &P = c->coef_host[p];
        const double hp = p > 0 ? hs(p - 1) : 0.0;
        const double hn = p < M ? hs(p) : 0.0;
        P.c1 = 0.5 * hp;
        P.c2 = 0.5 * hn;
        P.cL = P.c1;
        P.cR = P.c2;
        P.h = hn;
        P.t = ts(p);
        P.t_next = p < M ? ts(p + 1) : ts(M);
        P.dend = 0.0;
        P.traj = c->traj_rec ? c->traj_rec + 2 * p : nullptr;
        if (!self) {
            const double a = scale_at(c, P.t);
            P.ka1 = std::pow(a, 1.0 + al);
            P.ka3 = std::pow(a, 3.0 + al);
            P.dload = p > 0 ? hp * std::pow(scale_at(c, ts(p - 1) + 0.5 * hp), al - 3.0) : 0.0;
        }
    }
    if ((s = upload_coef(c, (size_t)M + 2)) != LAT_OK) return s;
    const int mode = self ? kLastSelf : kLastStore;
    s = launch_passes(c, dir * ns, M + 1, [&](hipStream_t st) {
        if (self) {
            hipLaunchKernelGGL(self_prologue, dim3(1), dim3(64), 0, st, c->coef, c->sc, al);
            HIPCHK(c, hipGetLastError());
        }
        for (int64_t p = 0; p <= M; ++p) {
            const int v = p == 0 ? (self ? kKickOnlyRed : kKickOnly) : (self ? kDriftKickRed : kDriftKick);
            const PassLink lk = self ? pass_link(c, p, kLastSelf, true) : PassLink{};
            lat_status r = run_pass(c, v, (int)p, mode, st, self ? &lk : nullptr);
            if (r != LAT_OK) return r;
        }
        return self ? finish_chain(c, M, kLastSelf, st) : LAT_OK;
    });
    if (s != LAT_OK) return s;
    c->t = t_start + (double)ns * h;
    return LAT_OK;
}

// energy pass + readback of the raw sums and the scale record
lat_status energy_sums(lat_ctx *c, double kick_c1)
{
    lat_status s = reserve_coef(c, 2);
    if (s != LAT_OK) return s;
    PassCoef &P = c->coef_host[0];
    const double a = scale_at(c, c->t);
    P.ka1 = std::pow(a, 1.0 + c->p.alpha);
    P.ka3 = std::pow(a, 3.0 + c->p.alpha);
    P.c1 = kick_c1;
    P.t = c->t;
    if ((s = upload_coef(c, 1)) != LAT_OK) return s;
    if (c->p.expansion == LAT_EXP_SELF && kick_c1 != 0.0) {
        hipLaunchKernelGGL(self_prologue, dim3(1), dim3(64), 0, c->stream, c->coef, c->sc, c->p.alpha);
        HIPCHK(c, hipGetLastError());
    }
    // the block sums go to a one-block kernel after the pass rather than to a
    // last block: no ticket release in the pass's blocks (LATTICE_ENERGY_DEFER=0
    // keeps the ticket; the same sums)
    const char *ed = std::getenv("LATTICE_ENERGY_DEFER");
    PassLink el;
    el.defer = 1;
    el.partials = c->partials;
    el.store_to = c->sc;
    if ((s = run_pass(c, kEnergy, 0, kLastStore, c->stream, (ed && std::atoi(ed) == 0) ? nullptr : &el)) != LAT_OK)
        return s;
    HIPCHK(c, hipMemcpyAsync(c->sc_host, c->sc, sizeof(ScaleRecord), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return LAT_OK;
}

bool aligned(const void *p, size_t a) { return ((uintptr_t)p % a) == 0; }

lat_status validate(const lat_params *p, const lat_fields *f)
{
    if (!p || !f) return fail(nullptr, LAT_EINVAL, "null params or fields");
    if (p->N < 2) return fail(nullptr, LAT_EINVAL, "N must be >= 2");
    if ((double)p->N * p->N * p->N > 4.0e10) return fail(nullptr, LAT_EINVAL, "N too large");
    if (!(p->dx > 0.0) || !std::isfinite(p->dx)) return fail(nullptr, LAT_EINVAL, "dx must be > 0");
    if (!(p->dt > 0.0) || !std::isfinite(p->dt)) return fail(nullptr, LAT_EINVAL, "dt must be > 0");
    if (p->dt / p->dx >= 1.0 / std::sqrt(3.0))
        return fail(nullptr, LAT_EINVAL, "dt/dx must be below 1/sqrt(3)");
    if (p->integrator < LAT_LF || p->integrator > LAT_VV10) return fail(nullptr, LAT_EINVAL, "bad integrator");
    if (p->expansion < LAT_EXP_NONE || p->expansion > LAT_EXP_SELF) return fail(nullptr, LAT_EINVAL, "bad expansion");
    if (p->potential < LAT_PHI4 || p->potential > LAT_SU2_HIGGS) return fail(nullptr, LAT_EINVAL, "bad potential");
    if (p->precision != LAT_PREC_F64 && p->precision != LAT_PREC_F32) return fail(nullptr, LAT_EINVAL, "bad precision");
    if (p->lf_staggered < -1 || p->lf_staggered > 1) return fail(nullptr, LAT_EINVAL, "lf_staggered must be -1, 0 or 1");
    if (p->lf_staggered != 0 && p->integrator != LAT_LF)
        return fail(nullptr, LAT_EINVAL, "lf_staggered needs the LF integrator");
    if (p->integrator == LAT_LF && p->expansion == LAT_EXP_SELF && p->lf_staggered != 0 && std::isnan(p->b0))
        return fail(nullptr, LAT_EINVAL, "a staggered leapfrog start with self-consistent expansion needs b0 "
                                         "(a' half a step behind)");
    if (p->expansion == LAT_EXP_FIXED) {
        const double den = 3.0 * (1.0 + p->w_eos) - 2.0 * p->alpha;
        if (den == 0.0 || !(p->a0 > 0.0)) return fail(nullptr, LAT_EINVAL, "bad fixed background");
    }
    if (p->expansion == LAT_EXP_SELF && !(p->a0 > 0.0)) return fail(nullptr, LAT_EINVAL, "a0 must be > 0");
    const size_t al = p->precision == LAT_PREC_F32 ? 4 : 8;
    const int nf = p->potential == LAT_PHI4 ? 1 : (p->potential == LAT_SU2_HIGGS ? 0 : 2);
    for (int i = 0; i < nf; ++i) {
        if (!f->phi[i] || !f->pi[i]) return fail(nullptr, LAT_EINVAL, "null field pointer");
        if (!aligned(f->phi[i], al) || !aligned(f->pi[i], al))
            return fail(nullptr, LAT_EINVAL, "misaligned field pointer");
    }
    if (p->potential == LAT_ABELIAN_HIGGS) {
        if (p->precision != LAT_PREC_F64) return fail(nullptr, LAT_EUNSUPPORTED, "the U(1) model runs in float64");
        if (!(p->e_charge != 0.0) || !(p->kappa_g > 0.0)) return fail(nullptr, LAT_EINVAL, "bad U(1) couplings");
        for (int i = 0; i < 3; ++i) {
            if (!f->A[i] || !f->piA[i]) return fail(nullptr, LAT_EINVAL, "null gauge field pointer");
            if (!aligned(f->A[i], al) || !aligned(f->piA[i], al))
                return fail(nullptr, LAT_EINVAL, "misaligned gauge field pointer");
        }
    }
    if (p->potential == LAT_SU2_HIGGS) {
        if (p->precision != LAT_PREC_F64) return fail(nullptr, LAT_EUNSUPPORTED, "the SU(2) model runs in float64");
        if (!(p->e_charge != 0.0) || !std::isfinite(p->e_charge)) return fail(nullptr, LAT_EINVAL, "bad SU(2) coupling");
        if ((double)p->N * p->N * p->N * 8.0 >= 4294967296.0)
            return fail(nullptr, LAT_EUNSUPPORTED, "the SU(2) model needs 8 N^3 < 2^32 (32-bit offsets)");
        const void *all[29];
        for (int k = 0; k < 4; ++k) {
            all[k] = f->doublet[k];
            all[4 + k] = f->pi_doublet[k];
        }
        for (int k = 0; k < 12; ++k) all[8 + k] = f->U[k];
        for (int k = 0; k < 9; ++k) all[20 + k] = f->E[k];
        for (const void *q : all) {
            if (!q) return fail(nullptr, LAT_EINVAL, "null SU(2) field pointer");
            if (!aligned(q, al)) return fail(nullptr, LAT_EINVAL, "misaligned SU(2) field pointer");
        }
    }
    return LAT_OK;
}

void free_ctx(lat_ctx *c)
{
    if (!c) return;
    (void)hipStreamSynchronize(c->stream);
    for (int f = 0; f < 2; ++f) {
        if (c->phi[f][1]) (void)hipFree(c->phi[f][1]);
        if (c->pi[f][1]) (void)hipFree(c->pi[f][1]);
    }
    for (int i = 0; i < 3; ++i)
        if (c->A[i][1]) (void)hipFree(c->A[i][1]);
    for (int k = 0; k < 4; ++k)
        if (c->dbl[k][1]) (void)hipFree(c->dbl[k][1]);
    for (int k = 0; k < 12; ++k)
        if (c->lnk[k][1]) (void)hipFree(c->lnk[k][1]);
    for (auto q : c->su2_aos)
        if (q) (void)hipFree(q);
    if (c->partials) (void)hipFree(c->partials);
    if (c->ticket) (void)hipFree(c->ticket);
    if (c->sc) (void)hipFree(c->sc);
    if (c->coef) (void)hipFree(c->coef);
    if (c->ring_base) (void)hipHostFree(c->ring_base);
    if (c->sc_host) (void)hipHostFree(c->sc_host);
    for (auto e : c->ring_ev)
        if (e) (void)hipEventDestroy(e);
    for (auto &t : c->timed) {
        (void)hipEventDestroy(t.start);
        (void)hipEventDestroy(t.stop);
    }
    for (auto e : c->spare) (void)hipEventDestroy(e);
    for (int k = 0; k < 2; ++k)
        for (int f = 0; f < 2; ++f)
            for (int b = 0; b < 2; ++b)
                if (c->lam[k][f][b]) (void)hipFree(c->lam[k][f][b]);
    if (c->ckpt) (void)hipFree(c->ckpt);
    if (c->adj_partials) (void)hipFree(c->adj_partials);
    if (c->self_seg) (void)hipFree(c->self_seg);
    if (c->self_part) (void)hipFree(c->self_part);
    if (c->self_traj) (void)hipFree(c->self_traj);
    if (c->graph_exec) (void)hipGraphExecDestroy(c->graph_exec);
    drop_step_graphs(c);
    if (c->graph) (void)hipGraphDestroy(c->graph);
    if (c->capture_stream) (void)hipStreamDestroy(c->capture_stream);
    if (c->reals_dev) (void)hipFree(c->reals_dev);
    if (c->block_work) (void)hipFree(c->block_work);
    for (int2 *t : c->seg_work) (void)hipFree(t);
    if (c->fft_plan) (void)hipfftDestroy(c->fft_plan);
    if (c->fft_inv) (void)hipfftDestroy(c->fft_inv);
    if (c->fft_in) (void)hipFree(c->fft_in);
    if (c->fft_out) (void)hipFree(c->fft_out);
    if (c->fft_out2) (void)hipFree(c->fft_out2);
    if (c->spec_part) (void)hipFree(c->spec_part);
    for (void *q : c->pi_scratch)
        if (q) (void)hipFree(q);
    for (lat_ctx *sub : c->subs) free_ctx(sub);
    delete c;
}

// ---------------------------------------------------------------------------
// allocation-free energies (lattice_energy_noalloc)
// ---------------------------------------------------------------------------
// Byte layout of the fixed per-GPU scratch array: the pass coefficients, the
// ticket counter, the record the last block writes the sums into, then the
// per-block partial sums.
constexpr size_t kNaCoef = 0, kNaTicket = 256, kNaRecord = 512, kNaPartials = 1024;
constexpr size_t kNaBytes = 512 * 1024 + kNaPartials;   // 513 KiB per GPU
constexpr size_t kNaPartialDoubles = (kNaBytes - kNaPartials) / sizeof(double);
constexpr int kNaMaxDevices = 64;
static_assert(sizeof(PassCoef) <= kNaTicket - kNaCoef && sizeof(ScaleRecord) <= kNaPartials - kNaRecord,
              "scratch layout");
static_assert(sizeof(scratch) == kNaBytes, "scratch size");

// coefficients of the read-only energy pass (kick on a copy by c1, no drift)
// and a cleared ticket; a kernel rather than a copy or a memset so that the
// call stays capturable into a HIP graph
__global__ void na_prepare(PassCoef *coef, unsigned *ticket, double ka1, double ka3, double c1, double t)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        PassCoef P{};
        P.ka1 = ka1;
        P.ka3 = ka3;
        P.c1 = c1;
        P.t = t;
        *coef = P;
        *ticket = 0u;
    }
}

// energies from the raw volume sums (eq. EK_EG_EV): out = EK[0], EK[1], EG[0],
// EG[1], EV[0], EV[1], rho, a
__global__ void na_finish(const ScaleRecord *sc, double *out, int nf, double inv_vol, double inv_dx2, double a)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        double rho = 0.0;
        for (int i = 0; i < 2; ++i) {
            const bool on = i < nf;
            const double ek = on ? sc->sums[i] * inv_vol / (2.0 * pow(a, 6.0)) : 0.0;
            const double eg = on ? sc->sums[nf + i] * inv_dx2 * inv_vol / (2.0 * a * a) : 0.0;
            const double ev = on ? sc->sums[2 * nf + i] * inv_vol : 0.0;
            out[i] = ek;
            out[2 + i] = eg;
            out[4 + i] = ev;
            rho += ek + eg + ev;
        }
        out[6] = rho;
        out[7] = a;
    }
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

const char *lattice_version(void) { return "paper_2102_01031_amd lattice 0.1 (gfx950)"; }

const char *lattice_last_error(const lat_ctx *ctx)
{
    return ctx ? ctx->err.c_str() : g_init_error.c_str();
}

lat_status lattice_init(lat_ctx **out, const lat_params *p, const lat_fields *f, void *stream)
{
    if (!out) return fail(nullptr, LAT_EINVAL, "null ctx pointer");
    *out = nullptr;
    lat_status s = validate(p, f);
    if (s != LAT_OK) return s;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return fail(nullptr, LAT_ENODEV, "no GPU available");

    lat_ctx *c = new (std::nothrow) lat_ctx();
    if (!c) return fail(nullptr, LAT_ENOMEM, "host allocation failed");
    c->p = *p;
    c->stream = (hipStream_t)stream;
    (void)hipGetDevice(&c->device);
    c->f32 = p->precision == LAT_PREC_F32;
    c->esize = c->f32 ? 4 : 8;
    c->u1 = p->potential == LAT_ABELIAN_HIGGS;
    c->su2 = p->potential == LAT_SU2_HIGGS;
    c->nf = p->potential == LAT_PHI4 ? 1 : (c->su2 ? 0 : 2);
    c->N = p->N;
    c->vol = (size_t)p->N * p->N * p->N;
    c->t = p->t0;
    c->lf_stag = p->lf_staggered;
    geometry_from_env(c);
    slab_config(c);
    energy_geometry(c);
    const size_t bytes = c->vol * c->esize;

    auto bail = [&](lat_status st, const std::string &m) {
        g_init_error = m;
        free_ctx(c);
        return st;
    };
    for (int i = 0; i < c->nf; ++i) {
        c->phi[i][0] = f->phi[i];
        c->pi[i][0] = f->pi[i];
        if (hipMalloc(&c->phi[i][1], bytes) != hipSuccess) return bail(LAT_ENOMEM, "shadow allocation failed");
        // U(1) momenta are read at their own site only and updated in place
        if (!c->u1 && hipMalloc(&c->pi[i][1], bytes) != hipSuccess)
            return bail(LAT_ENOMEM, "shadow allocation failed");
    }
    if (c->u1) {
        for (int i = 0; i < 3; ++i) {
            c->A[i][0] = f->A[i];
            c->piA[i] = f->piA[i];
            if (hipMalloc(&c->A[i][1], bytes) != hipSuccess) return bail(LAT_ENOMEM, "shadow allocation failed");
        }
    }
    if (c->su2) {
        for (int k = 0; k < 4; ++k) {
            c->dbl[k][0] = f->doublet[k];
            c->dpi[k] = f->pi_doublet[k];
            if (hipMalloc(&c->dbl[k][1], bytes) != hipSuccess) return bail(LAT_ENOMEM, "shadow allocation failed");
        }
        for (int k = 0; k < 12; ++k) {
            c->lnk[k][0] = f->U[k];
            if (hipMalloc(&c->lnk[k][1], bytes) != hipSuccess) return bail(LAT_ENOMEM, "shadow allocation failed");
        }
        for (int k = 0; k < 9; ++k) c->efl[k] = f->E[k];
        su2_geometry(c);
        // per-site records during multi-pass lattice_step calls (12% faster step
        // at 128^3); LATTICE_SU2_AOS=0 keeps the SoA arrays throughout
        const char *aenv = std::getenv("LATTICE_SU2_AOS");
        c->su2_aos_on = !(aenv && std::atoi(aenv) == 0) && (double)c->vol * 32.0 < 4294967296.0;
    }
    c->partial_cap = (size_t)std::max(c->nblocks > 1 ? c->nblocks : 1, c->en_nblocks) * kMaxQ + 64;
    if (c->su2) c->partial_cap = su2_partial_capacity(c->N) + 64;
    if (c->u1) {
        c->partial_cap = u1_partial_capacity(c->N) + 64;
        u1_geometry(c);
    }
    if (hipMalloc(&c->partials, c->partial_cap * sizeof(double)) != hipSuccess) return bail(LAT_ENOMEM, "scratch allocation failed");
    if (hipMalloc(&c->ticket, 64) != hipSuccess) return bail(LAT_ENOMEM, "scratch allocation failed");
    // the record, then two records for the deferred updates inside a call
    if (hipMalloc(&c->sc, 3 * sizeof(ScaleRecord)) != hipSuccess) return bail(LAT_ENOMEM, "scratch allocation failed");
    if (hipHostMalloc((void **)&c->sc_host, sizeof(ScaleRecord), hipHostMallocDefault) != hipSuccess)
        return bail(LAT_ENOMEM, "pinned allocation failed");
    for (auto &e : c->ring_ev)
        if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess)
            return bail(LAT_EHIP, "event creation failed");
    if (hipMemsetAsync(c->ticket, 0, 64, c->stream) != hipSuccess) return bail(LAT_EHIP, "memset failed");

    // initial scale record
    std::memset(c->sc_host, 0, sizeof(ScaleRecord));
    double a = 1.0, b = 0.0;
    if (p->expansion == LAT_EXP_FIXED) fixed_ab(*p, p->t0, &a, &b);
    if (p->expansion == LAT_EXP_SELF) {
        a = p->a0;
        b = p->b0;
    }
    c->sc_host->a = a;
    c->sc_host->b = std::isnan(b) ? 0.0 : b;
    c->sc_host->t = p->t0;
    if (hipMemcpyAsync(c->sc, c->sc_host, sizeof(ScaleRecord), hipMemcpyHostToDevice, c->stream) != hipSuccess)
        return bail(LAT_EHIP, "upload failed");
    if (hipStreamSynchronize(c->stream) != hipSuccess) return bail(LAT_EHIP, "stream synchronize failed");
    if (p->expansion == LAT_EXP_SELF && std::isnan(p->b0) && (c->u1 || c->su2)) {
        // Hubble constraint (eq. FriedmannHubble) with the gauge model's energies at a0
        lat_energies e{};
        if ((c->u1 ? u1_energy(c, &e) : su2_energy(c, &e)) != LAT_OK) return bail(LAT_EHIP, c->err);
        const double rhs = std::pow(a, 2.0 * p->alpha + 2.0) * p->kappa2 * e.rho / 3.0;
        if (!(rhs >= 0.0)) return bail(LAT_EINVAL, "negative energy: Hubble constraint has no root");
        c->sc_host->a = a;
        c->sc_host->b = std::sqrt(rhs);
        c->sc_host->t = p->t0;
        if (hipMemcpyAsync(c->sc, c->sc_host, sizeof(ScaleRecord), hipMemcpyHostToDevice, c->stream) != hipSuccess)
            return bail(LAT_EHIP, "upload failed");
        if (hipStreamSynchronize(c->stream) != hipSuccess) return bail(LAT_EHIP, "stream synchronize failed");
    } else if (p->expansion == LAT_EXP_SELF && std::isnan(p->b0)) {
        // Hubble constraint (eq. NewFriedmannEQsI): b0^2 = a0^{2 alpha + 2} kappa2 rho / 3
        if (energy_sums(c, 0.0) != LAT_OK) return bail(LAT_EHIP, c->err);
        const double *S = c->sc_host->sums;
        const int nf = c->nf;
        double sk = 0, sg = 0, sv = 0;
        for (int i = 0; i < nf; ++i) {
            sk += S[i];
            sg += S[nf + i];
            sv += S[2 * nf + i];
        }
        const double V = (double)c->vol;
        const double rho = sk / V / (2.0 * std::pow(a, 6.0)) + sg / (p->dx * p->dx) / V / (2.0 * a * a) + sv / V;
        const double rhs = std::pow(a, 2.0 * p->alpha + 2.0) * p->kappa2 * rho / 3.0;
        if (!(rhs >= 0.0)) return bail(LAT_EINVAL, "negative energy: Hubble constraint has no root");
        c->sc_host->a = a;
        c->sc_host->b = std::sqrt(rhs);
        c->sc_host->t = p->t0;
        if (hipMemcpyAsync(c->sc, c->sc_host, sizeof(ScaleRecord), hipMemcpyHostToDevice, c->stream) != hipSuccess)
            return bail(LAT_EHIP, "upload failed");
        if (hipStreamSynchronize(c->stream) != hipSuccess) return bail(LAT_EHIP, "stream synchronize failed");
    }
    if (p->expansion == LAT_EXP_SELF && p->integrator == LAT_LF && p->lf_staggered != 0 && !c->u1 && !c->su2) {
        // a staggered start: the next kick's b update needs the sums of the
        // stored half-step momenta squared (reading A3)
        if (energy_sums(c, 0.0) != LAT_OK) return bail(LAT_EHIP, c->err);
        for (int i = 0; i < c->nf; ++i) c->sc_host->sums[kPiPrev + i] = c->sc_host->sums[i];
        c->sc_host->a = a;
        c->sc_host->b = p->b0;
        c->sc_host->t = p->t0;
        if (hipMemcpyAsync(c->sc, c->sc_host, sizeof(ScaleRecord), hipMemcpyHostToDevice, c->stream) != hipSuccess)
            return bail(LAT_EHIP, "upload failed");
        if (hipStreamSynchronize(c->stream) != hipSuccess) return bail(LAT_EHIP, "stream synchronize failed");
    }
    *out = c;
    return LAT_OK;
}

lat_status lattice_step(lat_ctx *c, int64_t nsteps)
{
    if (!c) return fail(nullptr, LAT_EINVAL, "null context");
    if (nsteps == 0) return LAT_OK;
    const int dir = nsteps > 0 ? 1 : -1;
    const int64_t ns = nsteps > 0 ? nsteps : -nsteps;
    if (ns > (1LL << 30)) return fail(c, LAT_EINVAL, "too many steps in one call");
    lat_status s;
    if (c->p.integrator == LAT_LF && !c->batch && c->lf_stag != 0 && c->lf_stag != dir)
        return fail(c, LAT_ESTATE, "leapfrog momenta are staggered in the other direction; sync first");
    // A long call runs as consecutive calls of at most kChunkPasses stencil
    // passes, in chunks of equal length (+-1 step), so the per-call coefficient
    // tables, pinned staging and captured graphs stay bounded whatever the step
    // count; the result is bitwise that of the same steps issued as those
    // shorter calls.
    c->sums_fresh = false;
    const int64_t per = c->p.integrator == LAT_LF ? 1 : (int64_t)vv_weights(c->p.integrator).size();
    const int64_t cap = std::max<int64_t>(1, kChunkPasses / per);
    const int64_t nchunks = (ns + cap - 1) / cap;
    for (int64_t i = 0; i < nchunks; ++i) {
        const int64_t n = ns / nchunks + (i < ns % nchunks ? 1 : 0);
        if (c->batch) {
            if ((s = batch_step(c, dir * n)) != LAT_OK) return s;
            continue;
        }
        if (c->p.integrator == LAT_LF)
            s = c->su2 ? su2_step_lf(c, n, dir) : c->u1 ? u1_step_lf(c, n, dir) : step_lf(c, n, dir);
        else
            s = (c->u1 || c->su2) ? gauge_step_vv(c, n, dir) : step_vv(c, n, dir);
        if (s != LAT_OK) return s;
        if ((s = settle(c)) != LAT_OK) return s;
        c->step += dir * n;
    }
    // velocity-Verlet with self-consistent expansion: the call's last pass
    // reduced the energy sums of the state it leaves (momenta at integer time)
    c->sums_fresh = c->p.integrator != LAT_LF && c->p.expansion == LAT_EXP_SELF && !c->batch && !c->u1 && !c->su2;
    return LAT_OK;
}

lat_status lattice_sync(lat_ctx *c)
{
    if (!c) return fail(nullptr, LAT_EINVAL, "null context");
    if (c->batch) {
        for (lat_ctx *sub : c->subs) {
            lat_status st = lattice_sync(sub);
            if (st != LAT_OK) return fail(c, st, sub->err);
        }
        c->lf_stag = 0;
        return LAT_OK;
    }
    if (c->p.integrator != LAT_LF || c->lf_stag == 0) return LAT_OK;
    lat_status s;
    if (c->su2) {
        s = su2_sync(c);
    } else if (c->u1) {
        s = u1_sync(c);
    } else {
        if ((s = reserve_coef(c, 2)) != LAT_OK) return s;
        PassCoef &P = c->coef_host[0];
        const double a = scale_at(c, c->t);
        P.ka1 = std::pow(a, 1.0 + c->p.alpha);
        P.ka3 = std::pow(a, 3.0 + c->p.alpha);
        P.t = c->t;
        if (c->p.expansion == LAT_EXP_SELF) {
            // reading A3: b's half kick takes E_K of the momenta before the
            // kick (reduced with c1 = 0), the momenta kick by c2
            P.c1 = 0.0;
            P.c2 = 0.5 * c->lf_stag * c->p.dt;
            P.cL = 0.0;
            P.cR = 0.5 * c->lf_stag * c->p.dt;
            P.h = 0.0;
            P.t_next = c->t;
            if ((s = upload_coef(c, 2)) != LAT_OK) return s;
            hipLaunchKernelGGL(self_prologue, dim3(1), dim3(64), 0, c->stream, c->coef, c->sc, c->p.alpha);
            HIPCHK(c, hipGetLastError());
            s = run_pass(c, kKickOnlyRed, 0, kLastSelfLF);
        } else {
            P.c1 = 0.5 * c->lf_stag * c->p.dt;
            if ((s = upload_coef(c, 1)) != LAT_OK) return s;
            s = run_pass(c, kKickOnly, 0, kLastStore);
        }
    }
    if (s != LAT_OK) return s;
    if ((s = settle(c)) != LAT_OK) return s;
    c->lf_stag = 0;
    return LAT_OK;
}

lat_status lattice_energy(lat_ctx *c, lat_energies *out)
{
    if (!c || !out) return fail(c, LAT_EINVAL, "null argument");
    std::memset(out, 0, sizeof(*out));
    if (c->batch) return fail(c, LAT_EINVAL, "batch context: use lattice_energy_batch");
    if (c->u1) return u1_energy(c, out);
    if (c->su2) return su2_energy(c, out);
    const double c1 = (c->p.integrator == LAT_LF && c->lf_stag != 0) ? 0.5 * c->lf_stag * c->p.dt : 0.0;
    if (c->sums_fresh) {
        // the sums the last step call reduced at the state it left
        HIPCHK(c, hipMemcpyAsync(c->sc_host, c->sc, sizeof(ScaleRecord), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
    } else {
        lat_status s = energy_sums(c, c1);
        if (s != LAT_OK) return s;
    }
    double a = 1.0, b = 0.0;
    if (c->p.expansion == LAT_EXP_FIXED) fixed_ab(c->p, c->t, &a, &b);
    if (c->p.expansion == LAT_EXP_SELF) {
        a = c->sc_host->a;
        b = c->sc_host->b;
    }
    const double *S = c->sc_host->sums;
    const int nf = c->nf;
    const double V = (double)c->vol;
    double rho = 0.0, skh = 0.0, sg = 0.0, sv = 0.0;
    for (int i = 0; i < nf; ++i) {
        out->EK[i] = S[i] / V / (2.0 * std::pow(a, 6.0));
        out->EG[i] = S[nf + i] / (c->p.dx * c->p.dx) / V / (2.0 * a * a);
        out->EV[i] = S[2 * nf + i] / V;
        rho += out->EK[i] + out->EG[i] + out->EV[i];
        skh += S[kPiPrev + i];
        sg += S[nf + i];
        sv += S[2 * nf + i];
    }
    if (c->p.expansion == LAT_EXP_SELF && c->p.integrator == LAT_LF && c->lf_stag != 0) {
        // b at integer time: its half kick with E_K of the stored half-step
        // momenta (reading A3), not written back
        const double al = c->p.alpha;
        const double EK = skh / V / (2.0 * std::pow(a, 6.0));
        const double EG = sg / (c->p.dx * c->p.dx) / V / (2.0 * a * a);
        const double EV = sv / V;
        const double Ka = std::pow(a, 2.0 * al + 1.0) / 3.0 * c->p.kappa2 *
                          ((al - 2.0) * EK + al * EG + (al + 1.0) * EV);
        b += 0.5 * c->lf_stag * c->p.dt * Ka;
    }
    out->t = c->t;
    out->a = a;
    out->b = b;
    out->rho = rho;
    out->hubble_lhs = b * b;
    out->hubble_rhs = std::pow(a, 2.0 * c->p.alpha + 2.0) * c->p.kappa2 * rho / 3.0;
    const double den = out->hubble_lhs + out->hubble_rhs;
    out->hubble_res = den != 0.0 ? (out->hubble_lhs - out->hubble_rhs) / den : 0.0;
    out->step = c->step;
    return LAT_OK;
}

// Allocation-free energies of a real scalar state given directly (no
// context): the pass that lattice_energy launches, with its coefficients,
// ticket, sum record and block partials in the fixed per-GPU scratch array.
namespace {
std::mutex g_na_mu;
void *g_na_ptr[kNaMaxDevices] = {};

// address of this device's copy of the scratch array (looked up once per
// device, with that device current)
lat_status na_scratch(int dev, char **out)
{
    std::lock_guard<std::mutex> lk(g_na_mu);
    if (!g_na_ptr[dev]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(nullptr, LAT_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_na_ptr[dev] = ptr;
    }
    *out = (char *)g_na_ptr[dev];
    return LAT_OK;
}
}  // namespace

lat_status lattice_energy_noalloc(const lat_params *p, const lat_fields *f, double *out, void *stream)
{
    lat_status s = validate(p, f);
    if (s != LAT_OK) return s;
    if (p->potential != LAT_PHI4 && p->potential != LAT_PHI4_CHI2)
        return fail(nullptr, LAT_EUNSUPPORTED, "lattice_energy_noalloc takes the real scalar models");
    if (!out || !aligned(out, 8)) return fail(nullptr, LAT_EINVAL, "null or misaligned output pointer");
    // the stage passes' launch geometry lattice_init would choose (a host record
    // only; lattice_energy at N = 256 runs its pass in a geometry of its own)
    lat_ctx g;
    g.N = p->N;
    g.f32 = p->precision == LAT_PREC_F32;
    g.nf = p->potential == LAT_PHI4 ? 1 : 2;
    g.vol = (size_t)p->N * p->N * p->N;
    geometry_from_env(&g);
    const int NQ = 3 * g.nf;
    if ((size_t)g.nblocks * NQ > kNaPartialDoubles)
        return fail(nullptr, LAT_EINVAL,
                    "lattice too large for the fixed scratch of lattice_energy_noalloc (" +
                        std::to_string((size_t)g.nblocks * NQ) + " block partials, at most " +
                        std::to_string(kNaPartialDoubles) + ")");
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0) return fail(nullptr, LAT_ENODEV, "no current GPU");
    if (dev >= kNaMaxDevices) return fail(nullptr, LAT_EUNSUPPORTED, "device index beyond the scratch table");
    char *base = nullptr;
    if ((s = na_scratch(dev, &base)) != LAT_OK) return s;
    PassCoef *coef = (PassCoef *)(base + kNaCoef);
    unsigned *ticket = (unsigned *)(base + kNaTicket);
    ScaleRecord *rec = (ScaleRecord *)(base + kNaRecord);
    double *partials = (double *)(base + kNaPartials);

    // the scale factor and on-the-fly leapfrog half kick of lattice_energy on a
    // context just created with p
    double a = 1.0, b = 0.0;
    if (p->expansion == LAT_EXP_FIXED) fixed_ab(*p, p->t0, &a, &b);
    if (p->expansion == LAT_EXP_SELF) a = p->a0;
    const double c1 = (p->integrator == LAT_LF && p->lf_staggered != 0) ? 0.5 * p->lf_staggered * p->dt : 0.0;
    const hipStream_t st = (hipStream_t)stream;
    hipLaunchKernelGGL(na_prepare, dim3(1), dim3(64), 0, st, coef, ticket, std::pow(a, 1.0 + p->alpha),
                       std::pow(a, 3.0 + p->alpha), c1, p->t0);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(nullptr, LAT_EHIP, std::string("na_prepare: ") + hipGetErrorString(e));
    auto args = [&](auto *tag) {
        using T = std::remove_pointer_t<decltype(tag)>;
        ScalarArgs<T> A{};
        for (int i = 0; i < g.nf; ++i) {
            A.phi_in[i] = (const T *)f->phi[i];
            A.pi_in[i] = (const T *)f->pi[i];
        }
        A.N = g.N;
        A.zc = g.zc;
        A.tiles_x = g.tiles_x;
        A.tiles_y = g.tiles_y;
        A.y_fastest = g.rows_y_fastest;
        A.inv_dx2 = 1.0 / (p->dx * p->dx);
        A.lam = p->lambda;
        A.q = p->potential == LAT_PHI4_CHI2 ? p->q : 0.0;
        A.coef = coef;
        A.coef_next = coef;
        A.partials = partials;
        A.ticket = ticket;
        A.sc = rec;
        A.last_mode = kLastStore;
        A.alpha = p->alpha;
        A.kappa2 = p->kappa2;
        A.inv_vol = 1.0 / (double)g.vol;
        return A;
    };
    if (g.f32) {
        const ScalarArgs<float> A = args((float *)nullptr);
        e = g.rows ? (g.nf == 1 ? launch_rows<float, 1>(g.N, g.rows_ty, g.rows_pf, g.rows_vw, kEnergy, A, g.nblocks, st)
                                : launch_rows<float, 2>(g.N, g.rows_ty, g.rows_pf, g.rows_vw, kEnergy, A, g.nblocks, st))
                   : (g.nf == 1 ? launch_tile<float, 1>(g.tile, kEnergy, A, g.nblocks, st)
                                : launch_tile<float, 2>(g.tile, kEnergy, A, g.nblocks, st));
    } else {
        const ScalarArgs<double> A = args((double *)nullptr);
        e = g.rows ? (g.nf == 1 ? launch_rows<double, 1>(g.N, g.rows_ty, g.rows_pf, g.rows_vw, kEnergy, A, g.nblocks, st)
                                : launch_rows<double, 2>(g.N, g.rows_ty, g.rows_pf, g.rows_vw, kEnergy, A, g.nblocks, st))
                   : (g.nf == 1 ? launch_tile<double, 1>(g.tile, kEnergy, A, g.nblocks, st)
                                : launch_tile<double, 2>(g.tile, kEnergy, A, g.nblocks, st));
    }
    if (e != hipSuccess) return fail(nullptr, LAT_EHIP, std::string("energy pass: ") + hipGetErrorString(e));
    hipLaunchKernelGGL(na_finish, dim3(1), dim3(64), 0, st, rec, out, g.nf, 1.0 / (double)g.vol,
                       1.0 / (p->dx * p->dx), a);
    e = hipGetLastError();
    if (e != hipSuccess) return fail(nullptr, LAT_EHIP, std::string("na_finish: ") + hipGetErrorString(e));
    return LAT_OK;
}

// Power spectrum of one stored array (sec. 3.1, eq. discretePS): float64
// real-to-complex transform of the array (hipFFT), radial binning on the
// device, normalisation on the host.
constexpr int kSpecBlocks = 1024;

// Transform buffers and plans on first use (kept until lattice_destroy).
static lat_status ensure_fft(lat_ctx *c, bool inverse)
{
    const int N = c->N;
    const size_t V = c->vol, H = (size_t)N * N * (N / 2 + 1);
    if (!c->fft_in && hipMalloc(&c->fft_in, V * sizeof(double)) != hipSuccess) {
        c->fft_in = nullptr;
        return fail(c, LAT_ENOMEM, "spectrum buffers");
    }
    if (!c->fft_out && hipMalloc(&c->fft_out, H * sizeof(double2)) != hipSuccess) {
        c->fft_out = nullptr;
        return fail(c, LAT_ENOMEM, "spectrum buffers");
    }
    if (!c->spec_part &&
        hipMalloc(&c->spec_part, (size_t)4 * (kSpecBlocks + 1) * kSpecMaxBins * sizeof(double)) != hipSuccess) {
        c->spec_part = nullptr;
        return fail(c, LAT_ENOMEM, "spectrum buffers");
    }
    hipfftHandle *plan = inverse ? &c->fft_inv : &c->fft_plan;
    if (!*plan) {
        hipfftHandle h = nullptr;
        if (hipfftPlan3d(&h, N, N, N, inverse ? HIPFFT_Z2D : HIPFFT_D2Z) != HIPFFT_SUCCESS)
            return fail(c, LAT_EHIP, "hipfftPlan3d failed");
        *plan = h;
    }
    if (hipfftSetStream(*plan, c->stream) != HIPFFT_SUCCESS) return fail(c, LAT_EHIP, "hipfftSetStream failed");
    return LAT_OK;
}

// Weight of shell b >= 1 in eq. discretePS: k_b^3/(2 pi^2) (dx/N)^3 / (4 pi b^2),
// k_b = b k_IR, k_IR = 2 pi/(N dx).
static double shell_weight(int N, double dx, long b)
{
    const double pi = 3.14159265358979323846;
    const double kb = b * (2.0 * pi / (N * dx)), v = dx / N;
    return kb * kb * kb / (2.0 * pi * pi) * v * v * v / (4.0 * pi * (double)b * b);
}

// Copy (or widen) one stored array into the transform input and run the
// forward real-to-complex transform into out.
static lat_status forward_transform(lat_ctx *c, const void *src, double2 *out)
{
    const size_t V = c->vol;
    if (c->f32) {
        hipLaunchKernelGGL(widen_f32, dim3(1024), dim3(256), 0, c->stream, (const float *)src, c->fft_in, V);
        HIPCHK(c, hipGetLastError());
    } else {
        HIPCHK(c, hipMemcpyAsync(c->fft_in, src, V * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    }
    if (hipfftExecD2Z(c->fft_plan, c->fft_in, (hipfftDoubleComplex *)out) != HIPFFT_SUCCESS)
        return fail(c, LAT_EHIP, "hipfftExecD2Z failed");
    return LAT_OK;
}

lat_status lattice_gauss_init(lat_ctx *c, double *mean_charge)
{
    if (!c) return fail(nullptr, LAT_EINVAL, "null context");
    c->sums_fresh = false;
    if (c->batch) return fail(c, LAT_EINVAL, "batch context: use a single-lattice context");
    if (!c->su2 && !c->u1) return fail(c, LAT_EINVAL, "the Gauss law belongs to the U(1) and SU(2) models");
    lat_status st = ensure_fft(c, false);
    if (st != LAT_OK) return st;
    if ((st = ensure_fft(c, true)) != LAT_OK) return st;
    const int N = c->N;
    const size_t V = c->vol;
    const dim3 grid(1024), blk(256);
    int *flag = (int *)(c->ticket + 8);   // a word of the ticket block that no reduction uses
    const int ncol = c->su2 ? 3 : 1;
    double mean[3] = {0.0, 0.0, 0.0};
    // device copies of the SU(2) pointer tables
    struct Tables {
        const double *dbl[4], *dpi[4], *lnk[12];
    } tab{};
    Tables *tab_dev = nullptr;
    if (c->su2) {
        for (int k = 0; k < 4; ++k) {
            tab.dbl[k] = (const double *)c->dbl[k][c->cur_su2];
            tab.dpi[k] = (const double *)c->dpi[k];
        }
        for (int k = 0; k < 12; ++k) tab.lnk[k] = (const double *)c->lnk[k][c->cur_su2];
        tab_dev = (Tables *)c->spec_part;   // scratch: the spectrum partials are free between calls
        HIPCHK(c, hipMemcpyAsync(tab_dev, &tab, sizeof(tab), hipMemcpyHostToDevice, c->stream));
        HIPCHK(c, hipMemsetAsync(flag, 0, sizeof(int), c->stream));
    }
    for (int a = 0; a < ncol; ++a) {
        if (c->su2) {
            hipLaunchKernelGGL(gauss_charge_su2, grid, blk, 0, c->stream, (const double *const *)((char *)tab_dev + offsetof(Tables, dbl)),
                               (const double *const *)((char *)tab_dev + offsetof(Tables, dpi)), (const double *const *)((char *)tab_dev + offsetof(Tables, lnk)),
                               c->p.e_charge, a, V, c->fft_in, flag);
        } else {
            hipLaunchKernelGGL(gauss_charge_u1, grid, blk, 0, c->stream, (const double *)c->phi[0][c->cur_phi[0]],
                               (const double *)c->phi[1][c->cur_phi[1]], (const double *)c->pi[0][0],
                               (const double *)c->pi[1][0], c->p.e_charge * c->p.kappa_g, V, c->fft_in);
        }
        HIPCHK(c, hipGetLastError());
        if (hipfftExecD2Z(c->fft_plan, c->fft_in, (hipfftDoubleComplex *)c->fft_out) != HIPFFT_SUCCESS)
            return fail(c, LAT_EHIP, "hipfftExecD2Z failed");
        double2 zero{};
        HIPCHK(c, hipMemcpyAsync(&zero, c->fft_out, sizeof(double2), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        mean[a] = zero.x / (double)V;
        if (c->su2 && a == 0) {
            int bad = 0;
            HIPCHK(c, hipMemcpy(&bad, flag, sizeof(int), hipMemcpyDeviceToHost));
            if (bad) return fail(c, LAT_ESTATE, "the SU(2) Gauss solve needs the links at the identity");
        }
        hipLaunchKernelGGL(gauss_symbol, grid, blk, 0, c->stream, c->fft_out, N, c->p.dx);
        HIPCHK(c, hipGetLastError());
        if (hipfftExecZ2D(c->fft_inv, (hipfftDoubleComplex *)c->fft_out, c->fft_in) != HIPFFT_SUCCESS)
            return fail(c, LAT_EHIP, "hipfftExecZ2D failed");
        double *e[3];
        for (int i = 0; i < 3; ++i) e[i] = c->su2 ? (double *)c->efl[3 * i + a] : (double *)c->piA[i];
        hipLaunchKernelGGL(gauss_field, grid, blk, 0, c->stream, (const double *)c->fft_in, N,
                           1.0 / ((double)V * c->p.dx), e[0], e[1], e[2]);
        HIPCHK(c, hipGetLastError());
    }
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (mean_charge)
        for (int a = 0; a < ncol; ++a) mean_charge[a] = mean[a];
    return LAT_OK;
}

lat_status lattice_spectrum(lat_ctx *c, int32_t field, int32_t which, int32_t nbins, double *sum, double *delta,
                            int64_t *count)
{
    if (!c || !sum || !delta || !count) return fail(c, LAT_EINVAL, "null argument");
    if (c->batch) return fail(c, LAT_EINVAL, "batch context: use a single-lattice context");
    const int nfld = c->su2 ? 4 : (c->u1 ? 2 : c->nf);
    if (field < 0 || field >= nfld || (which != 0 && which != 1))
        return fail(c, LAT_EINVAL, "field or array out of range");
    if (nbins < 1 || nbins > kSpecMaxBins) return fail(c, LAT_EINVAL, "nbins out of range");
    const int N = c->N;
    const size_t V = c->vol, H = (size_t)N * N * (N / 2 + 1);
    lat_status st = ensure_fft(c, false);
    if (st != LAT_OK) return st;
    const void *src = which == 0 ? c->phi[field][c->cur_phi[field]] : c->pi[field][c->cur_pi[field]];
    if (c->su2) src = which == 0 ? c->dbl[field][c->cur_su2] : c->dpi[field];
    st = forward_transform(c, src, c->fft_out);
    if (st != LAT_OK) return st;
    const int nb = (int)std::min<size_t>(kSpecBlocks, (H + kSpecThreads - 1) / kSpecThreads);
    double *ps = c->spec_part, *pc = ps + (size_t)kSpecBlocks * kSpecMaxBins;
    double *tot = pc + (size_t)kSpecBlocks * kSpecMaxBins;
    hipLaunchKernelGGL(spectrum_bin, dim3(nb), dim3(kSpecThreads), 0, c->stream, c->fft_out, N, nbins, ps, pc);
    HIPCHK(c, hipGetLastError());
    hipLaunchKernelGGL(spectrum_reduce, dim3((nbins + 63) / 64), dim3(64), 0, c->stream, ps, pc, nb, nbins, tot,
                       tot + kSpecMaxBins);
    HIPCHK(c, hipGetLastError());
    std::vector<double> host(2 * (size_t)kSpecMaxBins);
    HIPCHK(c, hipMemcpyAsync(host.data(), tot, host.size() * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    for (int b = 0; b < nbins; ++b) {
        sum[b] = host[b];
        count[b] = (int64_t)std::llround(host[kSpecMaxBins + b]);
        delta[b] = b == 0 ? 0.0 : shell_weight(N, c->p.dx, b) * sum[b];
    }
    return LAT_OK;
}

// Lattice occupation number (eq. OccuppationNum) of one real scalar field:
// transforms of phi_s and pi_s, shell sums on the device, <phi^2> and <chi^2>
// for the effective mass by a fixed-order device reduction, normalisation on
// the host.
lat_status lattice_occupation(lat_ctx *c, int32_t field, int32_t nbins, double fstar2, double *n, int64_t *count)
{
    if (!c || !n || !count) return fail(c, LAT_EINVAL, "null argument");
    if (c->batch) return fail(c, LAT_EINVAL, "batch context: use a single-lattice context");
    if (c->u1 || c->su2) return fail(c, LAT_EUNSUPPORTED, "occupation numbers are defined for real scalar fields");
    if (field < 0 || field >= c->nf) return fail(c, LAT_EINVAL, "field out of range");
    if (nbins < 1 || nbins > kSpecMaxBins) return fail(c, LAT_EINVAL, "nbins out of range");
    if (!(fstar2 > 0.0) || !std::isfinite(fstar2)) return fail(c, LAT_EINVAL, "fstar2 must be positive");
    if (c->p.integrator == LAT_LF && c->lf_stag != 0)
        return fail(c, LAT_ESTATE, "momenta are at the half step: call lattice_sync first");
    const int N = c->N;
    const size_t V = c->vol, H = (size_t)N * N * (N / 2 + 1);
    lat_status st = ensure_fft(c, false);
    if (st != LAT_OK) return st;
    if (!c->fft_out2 && hipMalloc(&c->fft_out2, H * sizeof(double2)) != hipSuccess) {
        c->fft_out2 = nullptr;
        return fail(c, LAT_ENOMEM, "spectrum buffers");
    }
    // scale factor and its derivative at the current time
    double a = 1.0, b = 0.0;
    if (c->p.expansion == LAT_EXP_FIXED) fixed_ab(c->p, c->t, &a, &b);
    if (c->p.expansion == LAT_EXP_SELF) {
        HIPCHK(c, hipMemcpyAsync(c->sc_host, c->sc, sizeof(ScaleRecord), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        a = c->sc_host->a;
        b = c->sc_host->b;
    }
    st = forward_transform(c, c->phi[field][c->cur_phi[field]], c->fft_out);
    if (st != LAT_OK) return st;
    st = forward_transform(c, c->pi[field][c->cur_pi[field]], c->fft_out2);
    if (st != LAT_OK) return st;
    const size_t S = (size_t)kSpecBlocks * kSpecMaxBins;
    double *part = c->spec_part, *tot = part + 3 * S;
    double *sq_part = tot + 3 * kSpecMaxBins, *sq_tot = sq_part + 2 * kSpecBlocks;
    const int nb = (int)std::min<size_t>(kSpecBlocks, (H + kSpecThreads - 1) / kSpecThreads);
    hipLaunchKernelGGL(occupation_bin, dim3(nb), dim3(kSpecThreads), 0, c->stream, c->fft_out, c->fft_out2, N, nbins,
                       std::pow(a, c->p.alpha - 3.0), b / a, part, S);
    HIPCHK(c, hipGetLastError());
    hipLaunchKernelGGL(spectrum_reduce_q, dim3((nbins + 63) / 64, 3), dim3(64), 0, c->stream, part, S, nb, nbins, 3,
                       tot, kSpecMaxBins);
    HIPCHK(c, hipGetLastError());
    const int nq = (int)std::min<size_t>(kSpecBlocks, (V + kSpecThreads - 1) / kSpecThreads);
    const void *f0 = c->phi[0][c->cur_phi[0]], *f1 = c->nf > 1 ? c->phi[1][c->cur_phi[1]] : nullptr;
    if (c->f32)
        hipLaunchKernelGGL(sumsq_blocks<float>, dim3(nq), dim3(kSpecThreads), 0, c->stream, (const float *)f0,
                           (const float *)f1, V, sq_part);
    else
        hipLaunchKernelGGL(sumsq_blocks<double>, dim3(nq), dim3(kSpecThreads), 0, c->stream, (const double *)f0,
                           (const double *)f1, V, sq_part);
    HIPCHK(c, hipGetLastError());
    hipLaunchKernelGGL(sumsq_reduce, dim3(1), dim3(64), 0, c->stream, sq_part, nq, sq_tot);
    HIPCHK(c, hipGetLastError());
    std::vector<double> host(3 * (size_t)kSpecMaxBins + 2);
    HIPCHK(c, hipMemcpyAsync(host.data(), tot, 3 * kSpecMaxBins * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(host.data() + 3 * kSpecMaxBins, sq_tot, 2 * sizeof(double), hipMemcpyDeviceToHost,
                             c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    // <d^2V/dphi_s^2>: lambda/4 phi^4 -> 3 lambda phi^2; q/2 phi^2 chi^2 -> q chi^2 (phi), q phi^2 (chi)
    const double p2 = host[3 * kSpecMaxBins] / (double)V, c2 = host[3 * kSpecMaxBins + 1] / (double)V;
    double vpp = 0.0;
    if (field == 0) {
        vpp = 3.0 * c->p.lambda * p2;
        if (c->p.potential == LAT_PHI4_CHI2) vpp += c->p.q * c2;
    } else if (c->p.potential == LAT_PHI4_CHI2) {
        vpp = c->p.q * p2;
    }
    const double pi = 3.14159265358979323846;
    const double L = N * c->p.dx, N6 = (double)V * (double)V;
    const double pref = a * a * L * L * L / (2.0 * N6) * fstar2, wx = std::pow(a, 2.0 * (1.0 - c->p.alpha));
    for (int bin = 0; bin < nbins; ++bin) {
        count[bin] = (int64_t)std::llround(host[2 * kSpecMaxBins + bin]);
        if (bin == 0) {
            n[bin] = 0.0;
            continue;
        }
        const double kb = bin * (2.0 * pi / L);
        const double om = std::sqrt(kb * kb + a * a * vpp);
        n[bin] = pref * (om * host[bin] + wx * host[kSpecMaxBins + bin] / om) / (4.0 * pi * (double)bin * bin);
    }
    return LAT_OK;
}

lat_status lattice_profile(lat_ctx *c, int enable)
{
    if (!c) return fail(nullptr, LAT_EINVAL, "null context");
    c->profiling = enable != 0;
    return LAT_OK;
}

lat_status lattice_stats(lat_ctx *c, int reset, lat_stats *out)
{
    if (!c || !out) return fail(c, LAT_EINVAL, "null argument");
    lat_status s = harvest_timing(c);
    if (s != LAT_OK) return s;
    std::memset(out, 0, sizeof(*out));
    for (int i = 0; i < 8; ++i) {
        out->launches[i] = c->launches[i];
        out->kernel_ms[i] = c->kernel_ms[i];
    }
    out->blocks = c->nblocks;
    out->threads = c->rows ? 64 * c->rows_ty : kTiles[c->tile].tx * kTiles[c->tile].ty;
    out->tile_x = c->rows ? c->N : kTiles[c->tile].tx;
    out->tile_y = c->rows ? c->rows_ty : kTiles[c->tile].ty;
    out->z_chunk = c->zc;
    if (reset) {
        std::memset(c->launches, 0, sizeof(c->launches));
        std::memset(c->kernel_ms, 0, sizeof(c->kernel_ms));
    }
    return LAT_OK;
}

void lattice_destroy(lat_ctx *c) { free_ctx(c); }

}  // extern "C"

// ===========================================================================
// U(1) sector (a = 1, leapfrog)
// ===========================================================================
namespace {

constexpr int kU1TX = 64, kU1TY = 4;

size_t u1_partial_capacity(int N)
{
    const size_t tiles = (size_t)((N + kU1TX - 1) / kU1TX) * ((N + kU1TY - 1) / kU1TY) * (size_t)N;
    return tiles * (kU1Sums + kU1Maxes);
}

U1Args u1_args(lat_ctx *c, double ck, double hd, bool write_fields)
{
    U1Args a{};
    for (int i = 0; i < 2; ++i) {
        a.phi_in[i] = (const double *)c->phi[i][c->cur_phi[i]];
        a.phi_out[i] = write_fields ? (double *)c->phi[i][c->cur_phi[i] ^ 1] : nullptr;
        a.pi[i] = (double *)c->pi[i][0];
    }
    for (int i = 0; i < 3; ++i) {
        a.A_in[i] = (const double *)c->A[i][c->cur_A[i]];
        a.A_out[i] = write_fields ? (double *)c->A[i][c->cur_A[i] ^ 1] : nullptr;
        a.piA[i] = (double *)c->piA[i];
    }
    a.N = c->N;
    a.tiles_x = (c->N + kU1TX - 1) / kU1TX;
    a.tiles_y = (c->N + kU1TY - 1) / kU1TY;
    a.zc = c->u1_zc;
    a.dx = c->p.dx;
    a.e = c->p.e_charge;
    a.lam = c->p.lambda;
    a.v = c->p.v;
    a.kappa_g = c->p.kappa_g;
    a.ck = ck;
    a.hd = hd;
    a.la1 = a.la3 = a.lam1 = 1.0;
    a.hdA = hd;
    a.dw = nullptr;
    a.partials = c->partials;
    a.ticket = c->ticket;
    a.sc = c->sc;
    return a;
}

// the same in an expanding background: kick weights at scale factor ak, drift
// weights at the drift's midpoint am (sec. 5.5.2 kernels; reading R3)
U1Args u1_args_bg(lat_ctx *c, double ck, double h, double ak, double am, bool write_fields)
{
    U1Args a = u1_args(c, ck, h, write_fields);
    const double al = c->p.alpha;
    a.la1 = std::pow(ak, 1.0 + al);
    a.la3 = std::pow(ak, 3.0 + al);
    a.lam1 = std::pow(ak, al - 1.0);
    a.hd = h * std::pow(am, al - 3.0);
    a.hdA = h * std::pow(am, al - 1.0);
    return a;
}

// weights from the device record (self-consistent expansion)
U1Args u1_args_dev(lat_ctx *c, bool write_fields)
{
    U1Args a = u1_args(c, 0.0, 0.0, write_fields);
    a.dw = c->sc->w;
    return a;
}

U1SelfConst u1_self_const(const lat_ctx *c)
{
    return U1SelfConst{c->p.alpha, c->p.kappa2, 1.0 / (double)c->vol};
}

// whole-row leapfrog pass: N = 64 XS, rows per block TY in {4, 8} (N = 64)
// or {2, 4} (N = 128), 64 XS TY threads (one site each per plane)
bool u1_rows_shape_ok(int N, int ty)
{
    return (N == 64 && (ty == 4 || ty == 8)) || (N == 128 && (ty == 2 || ty == 4));
}

template <int MODE>
hipError_t launch_u1_rows(const lat_ctx *c, const U1Args &a)
{
    const int nb = (c->N / c->u1_ty) * ((c->N + c->u1_zc - 1) / c->u1_zc);
    const dim3 nt(c->N * c->u1_ty);
    if (c->N == 64 && c->u1_ty == 4) hipLaunchKernelGGL((u1_rows<1, 4, MODE>), dim3(nb), nt, 0, c->stream, a);
    else if (c->N == 64) hipLaunchKernelGGL((u1_rows<1, 8, MODE>), dim3(nb), nt, 0, c->stream, a);
    else if (c->u1_ty == 2) hipLaunchKernelGGL((u1_rows<2, 2, MODE>), dim3(nb), nt, 0, c->stream, a);
    else hipLaunchKernelGGL((u1_rows<2, 4, MODE>), dim3(nb), nt, 0, c->stream, a);
    return hipGetLastError();
}

// U(1) launch geometry: whole-row kernel for N = 64, 128 unless LATTICE_U1_TILE
// says "tile"; "TY,zc" overrides the row kernel's rows per block and z chunk.
void u1_geometry(lat_ctx *c)
{
    c->u1_rows = c->N == 64 || c->N == 128;
    c->u1_ty = 4;
    c->u1_zc = c->N == 128 ? 16 : 4;
    // the energy pass gives each block a column of z planes, about 256 blocks in
    // all: every block's ticket release writes back its XCD's L2, and these
    // releases queue per XCD (at 128^3: 337 us per pass in 8192 one-plane
    // blocks, 140 us at 8 planes, 114 us at 32 planes, 256 blocks).
    // LATTICE_U1_ENERGY_ZC overrides the planes per block.
    const long tpp = (long)((c->N + kU1TX - 1) / kU1TX) * ((c->N + kU1TY - 1) / kU1TY);
    c->u1_ezc = (int)std::min<long>(c->N, std::max<long>(1, ((long)c->N * tpp + 255) / 256));
    if (const char *ez = std::getenv("LATTICE_U1_ENERGY_ZC")) {
        const int v = std::atoi(ez);
        if (v >= 1 && v <= c->N) c->u1_ezc = v;
    }
    const char *env = std::getenv("LATTICE_U1_TILE");
    if (!env) return;
    if (std::strcmp(env, "tile") == 0) {
        c->u1_rows = false;
        return;
    }
    int ty = 0, zc = 0;
    if (c->u1_rows && std::sscanf(env, "%d,%d", &ty, &zc) == 2 && u1_rows_shape_ok(c->N, ty) && zc >= 1 &&
        zc <= c->N) {
        c->u1_ty = ty;
        c->u1_zc = zc;
    }
}

lat_status u1_launch(lat_ctx *c, int mode, const U1Args &a)
{
    const int nb = a.tiles_x * a.tiles_y * c->N;
    const int kind = 6;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    if (c->profiling) {
        lat_status st = timing_begin(c, &ev0, &ev1);
        if (st != LAT_OK) return st;
    }
    switch (mode) {
    case kU1Step:
        if (c->u1_rows) {
            HIPCHK(c, launch_u1_rows<kU1Step>(c, a));
            break;
        }
        hipLaunchKernelGGL((u1_stage<kU1TX, kU1TY, kU1Step>), dim3(nb), dim3(kU1TX * kU1TY), 0, c->stream, a);
        break;
    case kU1Kick:
        if (c->u1_rows) {
            HIPCHK(c, launch_u1_rows<kU1Kick>(c, a));
            break;
        }
        hipLaunchKernelGGL((u1_stage<kU1TX, kU1TY, kU1Kick>), dim3(nb), dim3(kU1TX * kU1TY), 0, c->stream, a);
        break;
    case kU1Drift:
        hipLaunchKernelGGL(u1_drift, dim3((unsigned)((c->vol + 255) / 256)), dim3(256), 0, c->stream, a,
                           (unsigned)c->vol);
        break;
    default: {   // the summing passes: energy, kick and sums (row kernel only)
        U1Args e = a;
        e.defer = gauge_defer_on() ? 1 : 0;
        int fnt, fnb;
        if (c->u1_rows) {
            HIPCHK(c, mode == kU1KickSums ? launch_u1_rows<kU1KickSums>(c, e) : launch_u1_rows<kU1Energy>(c, e));
            fnt = c->N * c->u1_ty;
            fnb = (c->N / c->u1_ty) * ((c->N + c->u1_zc - 1) / c->u1_zc);
        } else {
            if (mode == kU1KickSums) return fail(c, LAT_EINVAL, "U(1) kick-and-sums pass needs the row kernel");
            e.zc = c->u1_ezc;
            fnb = a.tiles_x * a.tiles_y * ((c->N + e.zc - 1) / e.zc);
            fnt = kU1TX * kU1TY;
            hipLaunchKernelGGL((u1_stage<kU1TX, kU1TY, kU1Energy>), dim3(fnb), dim3(fnt), 0, c->stream, e);
        }
        HIPCHK(c, hipGetLastError());
        if (e.defer) HIPCHK(c, launch_gauge_sums_finish(fnt, e.partials, fnb, e.sc, c->stream));
        break;
    }
    }
    HIPCHK(c, hipGetLastError());
    if (c->profiling) {
        lat_status st = timing_end(c, ev0, ev1, kind);
        if (st != LAT_OK) return st;
    }
    c->launches[kind] += 1;
    return LAT_OK;
}

lat_status u1_flip(lat_ctx *c)
{
    for (int i = 0; i < 2; ++i) c->cur_phi[i] ^= 1;
    for (int i = 0; i < 3; ++i) c->cur_A[i] ^= 1;
    return LAT_OK;
}

#define U1K(kernel, ...)                                                            \
    do {                                                                            \
        hipLaunchKernelGGL(kernel, dim3(1), dim3(64), 0, c->stream, __VA_ARGS__);   \
        HIPCHK(c, hipGetLastError());                                               \
    } while (0)

// LATTICE_U1_FUSE=0 turns off the shortcuts of the self-consistent gauge steps
// (the U(1) kick pass that also forms the sums and the U(1) drift-only pass,
// bit for bit the same results; the SU(2) drift-only pass, the same to rounding).
static bool u1_fuse_on()
{
    const char *e = std::getenv("LATTICE_U1_FUSE");
    return e ? std::atoi(e) != 0 : true;
}

// The drift with the record's weights (its kick weight is zero): u1_drift in
// place of a step pass.
lat_status u1_drift_pass(lat_ctx *c)
{
    const bool drift = u1_fuse_on() && c->vol <= 0xffffffffu;   // 32-bit site index
    return u1_launch(c, drift ? kU1Drift : kU1Step, u1_args_dev(c, true));
}

// The kick with the record's weights followed by the volume sums of the kicked
// state (the b kick's "after" sums): one row-kernel pass where the row kernel
// runs, which forms the sums an energy pass with zero kick weight would, bit for
// bit.
lat_status u1_kick_sums(lat_ctx *c)
{
    if (c->u1_rows && u1_fuse_on()) return u1_launch(c, kU1KickSums, u1_args_dev(c, false));
    lat_status s = u1_launch(c, kU1Kick, u1_args_dev(c, false));
    if (s != LAT_OK) return s;
    return u1_launch(c, kU1Energy, u1_args(c, 0.0, 0.0, false));
}

// Leapfrog steps of the self-consistent gauge models after a call's first take
// the sums before the kick from the neighbouring passes (u1_self_drift_w) in
// place of an energy pass of their own; LATTICE_SELF_CARRY=0 measures them on
// every step (the same values).
static bool self_carry()
{
    const char *e = std::getenv("LATTICE_SELF_CARRY");
    return e ? std::atoi(e) != 0 : true;
}

// Self-consistent expansion (readings A3 and R1 for the U(1) model): the kicks,
// energy sums and drifts as separate passes, the scale factor, b and the pass
// weights updated on the device between them (stage_u1.hpp, U1SelfConst).
lat_status u1_step_self_lf(lat_ctx *c, int64_t ns, int dir)
{
    const double h = dir * c->p.dt;
    const U1SelfConst kc = u1_self_const(c);
    int stag = c->lf_stag;
    lat_status s;
    const bool carry_on = self_carry();
    for (int64_t k = 0; k < ns; ++k) {
        const double w = stag == 0 ? 0.5 * h : h;
        // sums of the state before the kick: measured on a call's first step,
        // carried from the passes around it on the later ones
        const int carry = stag != 0 && k > 0 && carry_on;
        if (stag != 0 && !carry) {
            if ((s = u1_launch(c, kU1Energy, u1_args(c, 0.0, 0.0, false))) != LAT_OK) return s;
            U1K(u1_self_stash, c->sc);
        }
        U1K(u1_self_kick_w, c->sc, w, c->p.alpha);
        if ((s = u1_kick_sums(c)) != LAT_OK) return s;
        U1K(u1_self_drift_w, c->sc, h, stag == 0 ? 0.0 : 0.5 * h, stag == 0 ? w : 0.5 * h, kc, carry);
        if ((s = u1_drift_pass(c)) != LAT_OK) return s;
        u1_flip(c);
        stag = dir;
    }
    c->lf_stag = dir;
    c->t += (double)ns * h;
    return LAT_OK;
}

lat_status u1_step_lf(lat_ctx *c, int64_t ns, int dir)
{
    if (c->p.expansion == LAT_EXP_SELF) return u1_step_self_lf(c, ns, dir);
    const double h = dir * c->p.dt;
    const double t0 = c->t;
    int stag = c->lf_stag;
    for (int64_t k = 0; k < ns; ++k) {
        const double ck = stag == 0 ? 0.5 * h : h;
        const double t = t0 + (double)k * h;
        lat_status s = u1_launch(c, kU1Step, c->p.expansion == LAT_EXP_FIXED
                                                 ? u1_args_bg(c, ck, h, scale_at(c, t), scale_at(c, t + 0.5 * h), true)
                                                 : u1_args(c, ck, h, true));
        if (s != LAT_OK) return s;
        u1_flip(c);
        stag = dir;
    }
    c->lf_stag = dir;
    c->t = t0 + (double)ns * h;
    return LAT_OK;
}

lat_status u1_sync(lat_ctx *c)
{
    const double w = 0.5 * c->lf_stag * c->p.dt;
    if (c->p.expansion == LAT_EXP_SELF) {
        lat_status s = u1_launch(c, kU1Energy, u1_args(c, 0.0, 0.0, false));
        if (s != LAT_OK) return s;
        U1K(u1_self_b_kick, c->sc, w, u1_self_const(c));
        U1K(u1_self_kick_w, c->sc, w, c->p.alpha);
        return u1_launch(c, kU1Kick, u1_args_dev(c, false));
    }
    const double a = scale_at(c, c->t);
    return u1_launch(c, kU1Kick, u1_args_bg(c, w, 0.0, a, a, false));
}

lat_status u1_energy(lat_ctx *c, lat_energies *out)
{
    const double ck = c->lf_stag != 0 ? 0.5 * c->lf_stag * c->p.dt : 0.0;
    const double V = (double)c->vol, al = c->p.alpha;
    double a = 1.0, b = 0.0;
    lat_status s;
    if (c->p.expansion == LAT_EXP_FIXED) fixed_ab(c->p, c->t, &a, &b);
    if (c->p.expansion == LAT_EXP_SELF) {
        // a and b of the record; a staggered b is half-kicked on the fly with
        // the sums of the stored half-step momenta (reading A3)
        if (ck != 0.0 && (s = u1_launch(c, kU1Energy, u1_args(c, 0.0, 0.0, false))) != LAT_OK) return s;
        HIPCHK(c, hipMemcpyAsync(c->sc_host, c->sc, sizeof(ScaleRecord), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        a = c->sc_host->a;
        b = c->sc_host->b;
        if (ck != 0.0) {
            const double *S = c->sc_host->sums;
            const double a2 = a * a, a4 = a2 * a2, a6 = a4 * a2;
            const double Ka = std::pow(a, 2.0 * al + 1.0) / 3.0 * c->p.kappa2 *
                              ((al - 2.0) * S[0] / V / a6 + al * S[1] / V / a2 +
                               (al - 1.0) * (S[3] / V / a4 + S[4] / V / a4) + (al + 1.0) * S[2] / V);
            b += ck * Ka;
        }
    }
    s = u1_launch(c, kU1Energy, u1_args_bg(c, ck, 0.0, a, a, false));
    if (s != LAT_OK) return s;
    HIPCHK(c, hipMemcpyAsync(c->sc_host, c->sc, sizeof(ScaleRecord), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    const double *S = c->sc_host->sums, *M = c->sc_host->maxes;
    const double a2 = a * a, a4 = a2 * a2, a6 = a4 * a2;
    out->t = c->t;
    out->a = a;
    out->b = b;
    out->EK[0] = S[0] / V / a6;
    out->EG[0] = S[1] / V / a2;
    out->EV[0] = S[2] / V;
    out->EK_A = S[3] / V / a4;
    out->EG_A = S[4] / V / a4;
    out->rho = out->EK[0] + out->EG[0] + out->EV[0] + out->EK_A + out->EG_A;
    out->hubble_lhs = b * b;
    out->hubble_rhs = std::pow(a, 2.0 * al + 2.0) * c->p.kappa2 * out->rho / 3.0;
    {
        const double den = out->hubble_lhs + out->hubble_rhs;
        out->hubble_res = den != 0.0 ? (out->hubble_lhs - out->hubble_rhs) / den : 0.0;
    }
    out->gauss_mean = S[5] / V;
    out->gauss_sum_mean = S[6] / V;
    out->gauss_abs_mean = S[7] / V;
    out->gauss_max = M[0];
    out->gauss_div_max = M[1];
    out->gauss_charge_max = M[2];
    out->step = c->step;
    return LAT_OK;
}

}  // namespace

// ===========================================================================
// SU(2) doublet + links (a = 1, leapfrog)
// ===========================================================================
namespace {

constexpr int kSU2TX = 64, kSU2TY = 4;

size_t su2_partial_capacity(int N)
{
    // largest grid: one z plane per block
    const size_t tiles = (size_t)((N + kSU2TX - 1) / kSU2TX) * ((N + kSU2TY - 1) / kSU2TY) * (size_t)N;
    return tiles * (kSU2Sums + kSU2Maxes);
}

// SU(2) block order, z planes per block and cache policy.  With N a multiple
// of 32 each XCD takes a y band of tiles_y / 8 tiles over all planes, one
// plane per block, so the blocks an XCD runs at once form a compact region
// whose neighbour planes stay in its L2 (LATTICE_SU2_BAND=0: the plane-wide
// order, in which an XCD's blocks march whole planes).  LATTICE_SU2_ZC
// overrides the planes per block.  The step passes read and write the
// momenta and write the output records non-temporally (LATTICE_SU2_NT=0:
// through the caches), which keeps the input records in L2.  At 128^3 on
// one GPU: 286.7 us per pass plane-wide, 236.7-240.1 in bands, 227.6-228.0
// in bands with the streams non-temporal.
void su2_geometry(lat_ctx *c)
{
    const int ty = (c->N + kSU2TY - 1) / kSU2TY;
    const char *e = std::getenv("LATTICE_SU2_BAND");
    c->su2_band = (ty % 8 == 0 && !(e && std::atoi(e) == 0)) ? ty / 8 : 0;
    c->su2_zc = su2_zc(c->N, c->su2_band > 0);
    const char *nt = std::getenv("LATTICE_SU2_NT");
    c->su2_nt = (nt && std::atoi(nt) == 0) ? 0 : 1;
}

// z planes per block: LATTICE_SU2_ZC if set (1 .. N), else 1 in the band
// order and otherwise a default that keeps at least 512 blocks
int su2_zc(int N, bool band)
{
    const char *env = std::getenv("LATTICE_SU2_ZC");
    int zc = 0;
    if (env && std::sscanf(env, "%d", &zc) == 1 && zc >= 1 && zc <= N) return zc;
    if (band) return 1;
    const int tiles = ((N + kSU2TX - 1) / kSU2TX) * ((N + kSU2TY - 1) / kSU2TY);
    zc = 16;
    while (zc > 1 && (size_t)tiles * ((N + zc - 1) / zc) < 512) zc /= 2;
    return zc;
}

SU2Args su2_args(lat_ctx *c, double ck, double hd, bool write_fields)
{
    SU2Args a{};
    const int cur = c->cur_su2;
    for (int k = 0; k < 4; ++k) {
        a.phi_in[k] = (const double *)c->dbl[k][cur];
        a.phi_out[k] = write_fields ? (double *)c->dbl[k][cur ^ 1] : nullptr;
        a.pi[k] = (double *)c->dpi[k];
    }
    for (int k = 0; k < 12; ++k) {
        a.U_in[k] = (const double *)c->lnk[k][cur];
        a.U_out[k] = write_fields ? (double *)c->lnk[k][cur ^ 1] : nullptr;
    }
    for (int k = 0; k < 9; ++k) a.E[k] = (double *)c->efl[k];
    a.N = c->N;
    a.tiles_x = (c->N + kSU2TX - 1) / kSU2TX;
    a.tiles_y = (c->N + kSU2TY - 1) / kSU2TY;
    a.zc = c->su2_zc;
    a.band = c->su2_band;
    a.dx = c->p.dx;
    a.g = c->p.e_charge;
    a.lam = c->p.lambda;
    a.v = c->p.v;
    a.ck = ck;
    a.hd = hd;
    a.la1 = a.la3 = a.lam1 = 1.0;
    a.hdU = hd;
    a.dw = nullptr;
    a.partials = c->partials;
    a.ticket = c->ticket;
    a.sc = c->sc;
    return a;
}

// expanding background: kick weights at scale factor ak, drift weights at the
// drift's midpoint am (sec. 5.5.2 kernels; reading R3)
void su2_bg(const lat_ctx *c, SU2Args &a, double h, double ak, double am)
{
    const double al = c->p.alpha;
    a.la1 = std::pow(ak, 1.0 + al);
    a.la3 = std::pow(ak, 3.0 + al);
    a.lam1 = std::pow(ak, al - 1.0);
    a.hd = h * std::pow(am, al - 3.0);
    a.hdU = h * std::pow(am, al - 1.0);
}

SU2Args su2_args_bg(lat_ctx *c, double ck, double h, double ak, double am, bool write_fields)
{
    SU2Args a = su2_args(c, ck, h, write_fields);
    su2_bg(c, a, h, ak, am);
    return a;
}

// weights from the device record (self-consistent expansion)
SU2Args su2_args_dev(lat_ctx *c, bool write_fields)
{
    SU2Args a = su2_args(c, 0.0, 0.0, write_fields);
    a.dw = c->sc->w;
    return a;
}

lat_status su2_launch(lat_ctx *c, int mode, const SU2Args &args)
{
    // the energy pass keeps the plane-wide order with its z columns: in the
    // band order's one-plane blocks its last block would sum 16x more block
    // partials (654 against 357 us at 128^3)
    SU2Args a = args;
    const bool sums = mode == kSU2Energy || mode == kSU2KickSums;
    if (sums) {
        a.band = 0;
        a.zc = su2_zc(c->N, false);
        a.defer = gauge_defer_on() ? 1 : 0;
        // LATTICE_SU2_ENERGY_ZC: z planes per block of the summing passes alone
        if (const char *ez = std::getenv("LATTICE_SU2_ENERGY_ZC")) {
            const int v = std::atoi(ez);
            if (v >= 1 && v <= c->N) a.zc = v;
        }
    }
    const size_t nbz = (size_t)a.tiles_x * a.tiles_y * (size_t)((c->N + a.zc - 1) / a.zc);
    if (nbz > 0x7fffffffu || (sums && nbz * (kSU2Sums + kSU2Maxes) > c->partial_cap))
        return fail(c, LAT_EINVAL, "SU(2) launch exceeds the partials buffer");
    const int nb = (int)nbz;
    const int kind = 6;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    if (c->profiling) {
        lat_status st = timing_begin(c, &ev0, &ev1);
        if (st != LAT_OK) return st;
    }
    const dim3 grid(nb), blk(kSU2TX * kSU2TY);
    const bool nt = c->su2_nt != 0;
    switch (mode) {
    case kSU2Drift:
        hipLaunchKernelGGL(su2_drift, dim3((unsigned)((c->vol + 255) / 256)), dim3(256), 0, c->stream, a,
                           (unsigned)c->vol);
        break;
    case kSU2Step:
        if (nt) hipLaunchKernelGGL((su2_stage<kSU2TX, kSU2TY, kSU2Step, true>), grid, blk, 0, c->stream, a);
        else hipLaunchKernelGGL((su2_stage<kSU2TX, kSU2TY, kSU2Step, false>), grid, blk, 0, c->stream, a);
        break;
    case kSU2Kick: hipLaunchKernelGGL((su2_stage<kSU2TX, kSU2TY, kSU2Kick, false>), grid, blk, 0, c->stream, a); break;
    case kSU2KickSums:
        hipLaunchKernelGGL((su2_stage<kSU2TX, kSU2TY, kSU2KickSums, false>), grid, blk, 0, c->stream, a);
        HIPCHK(c, hipGetLastError());
        if (a.defer) HIPCHK(c, launch_gauge_sums_finish(kSU2TX * kSU2TY, a.partials, nb, a.sc, c->stream));
        break;
    case kSU2StepAoS:
        if (nt) hipLaunchKernelGGL((su2_stage<kSU2TX, kSU2TY, kSU2StepAoS, true>), grid, blk, 0, c->stream, a);
        else hipLaunchKernelGGL((su2_stage<kSU2TX, kSU2TY, kSU2StepAoS, false>), grid, blk, 0, c->stream, a);
        break;
    default:
        hipLaunchKernelGGL((su2_stage<kSU2TX, kSU2TY, kSU2Energy, false>), grid, blk, 0, c->stream, a);
        HIPCHK(c, hipGetLastError());
        if (a.defer) HIPCHK(c, launch_gauge_sums_finish(kSU2TX * kSU2TY, a.partials, nb, a.sc, c->stream));
        break;
    }
    HIPCHK(c, hipGetLastError());
    if (c->profiling) {
        lat_status st = timing_end(c, ev0, ev1, kind);
        if (st != LAT_OK) return st;
    }
    c->launches[kind] += 1;
    return LAT_OK;
}

// Per-site records: buffers on first use, conversion from / to the SoA arrays
// of the current parity (from: back into the caller's arrays, parity 0).  A
// call converts twice, so records are used from this many passes on.
constexpr int64_t kSU2AosMinPasses = 4;
lat_status su2_aos_enter(lat_ctx *c)
{
    for (auto &q : c->su2_aos)
        if (!q && hipMalloc(&q, 4 * c->vol * sizeof(double4)) != hipSuccess) {
            q = nullptr;
            return fail(c, LAT_ENOMEM, "SU(2) record buffers");
        }
    SU2Soa s{};
    for (int k = 0; k < 4; ++k) s.a[k] = (double *)c->dbl[k][c->cur_su2];
    for (int k = 0; k < 12; ++k) s.a[4 + k] = (double *)c->lnk[k][c->cur_su2];
    SU2Aos d{};
    for (int q = 0; q < 4; ++q) d.r[q] = c->su2_aos[0] + (size_t)q * c->vol;
    hipLaunchKernelGGL(su2_to_aos, dim3(2048), dim3(256), 0, c->stream, s, d, c->vol);
    HIPCHK(c, hipGetLastError());
    return LAT_OK;
}

lat_status su2_aos_leave(lat_ctx *c, int buf)
{
    SU2Aos s{};
    for (int q = 0; q < 4; ++q) s.r[q] = c->su2_aos[buf] + (size_t)q * c->vol;
    SU2Soa d{};
    for (int k = 0; k < 4; ++k) d.a[k] = (double *)c->dbl[k][0];
    for (int k = 0; k < 12; ++k) d.a[4 + k] = (double *)c->lnk[k][0];
    hipLaunchKernelGGL(su2_from_aos, dim3(2048), dim3(256), 0, c->stream, s, d, c->vol);
    HIPCHK(c, hipGetLastError());
    c->cur_su2 = 0;
    return LAT_OK;
}

SU2Args su2_args_aos(lat_ctx *c, double ck, double hd, int buf)
{
    SU2Args a = su2_args(c, ck, hd, false);
    const double4 *in = c->su2_aos[buf];
    double4 *out = c->su2_aos[buf ^ 1];
    a.phi_in4 = in;
    a.phi_out4 = out;
    for (int i = 0; i < 3; ++i) {
        a.U_in4[i] = in + (size_t)(1 + i) * c->vol;
        a.U_out4[i] = out + (size_t)(1 + i) * c->vol;
    }
    return a;
}

// Leapfrog passes alternate the z march direction of every column (odd
// passes of a call march down), so a pass starts on the planes the pass
// before it wrote last, which the memory-side cache still holds; each site's
// update is independent of the order.  Measured 297 -> 287 us per 128^3 pass
// on records.  LATTICE_SU2_ALT=0 keeps upward marches.
static bool su2_alternate()
{
    const char *e = std::getenv("LATTICE_SU2_ALT");
    return e ? std::atoi(e) != 0 : true;
}

// Self-consistent expansion (readings A3 and R1 for the SU(2) model), as the
// U(1) model's: the kicks, energy sums and drifts as separate passes on the
// plain arrays, the scale factor, b and the pass weights updated on the device
// between them with the U(1) model's one-thread kernels (the SU(2) energy pass
// leaves its sums in the same slots: doublet kinetic, gradient, potential,
// electric, magnetic).
// The drift with the record's weights (its kick weight is zero): su2_drift in
// place of a step pass (the same values to rounding); LATTICE_U1_FUSE=0 runs
// the step pass, as for the U(1) model.
lat_status su2_drift_pass(lat_ctx *c)
{
    const bool drift = u1_fuse_on() && c->vol <= 0xffffffffu;
    return su2_launch(c, drift ? kSU2Drift : kSU2Step, su2_args_dev(c, true));
}

// The kick with the record's weights followed by the volume sums of the kicked
// state: one pass in the energy pass's launch shape (kSU2KickSums) forming the
// sums that pass would; LATTICE_U1_FUSE=0 runs the two passes.
lat_status su2_kick_sums(lat_ctx *c)
{
    if (u1_fuse_on()) return su2_launch(c, kSU2KickSums, su2_args_dev(c, false));
    lat_status s = su2_launch(c, kSU2Kick, su2_args_dev(c, false));
    if (s != LAT_OK) return s;
    return su2_launch(c, kSU2Energy, su2_args(c, 0.0, 0.0, false));
}

lat_status su2_step_self_lf(lat_ctx *c, int64_t ns, int dir)
{
    const double h = dir * c->p.dt;
    const U1SelfConst kc = u1_self_const(c);
    int stag = c->lf_stag;
    lat_status s;
    const bool carry_on = self_carry();
    for (int64_t k = 0; k < ns; ++k) {
        const double w = stag == 0 ? 0.5 * h : h;
        const int carry = stag != 0 && k > 0 && carry_on;   // as in u1_step_self_lf
        if (stag != 0 && !carry) {
            if ((s = su2_launch(c, kSU2Energy, su2_args(c, 0.0, 0.0, false))) != LAT_OK) return s;
            U1K(u1_self_stash, c->sc);
        }
        U1K(u1_self_kick_w, c->sc, w, c->p.alpha);
        if ((s = su2_kick_sums(c)) != LAT_OK) return s;
        U1K(u1_self_drift_w, c->sc, h, stag == 0 ? 0.0 : 0.5 * h, stag == 0 ? w : 0.5 * h, kc, carry);
        if ((s = su2_drift_pass(c)) != LAT_OK) return s;
        c->cur_su2 ^= 1;
        stag = dir;
    }
    c->lf_stag = dir;
    c->t += (double)ns * h;
    return LAT_OK;
}

lat_status su2_step_lf(lat_ctx *c, int64_t ns, int dir)
{
    if (c->p.expansion == LAT_EXP_SELF) return su2_step_self_lf(c, ns, dir);
    const double h = dir * c->p.dt;
    const double t0 = c->t;
    const bool fixed = c->p.expansion == LAT_EXP_FIXED;
    int stag = c->lf_stag;
    if (c->su2_aos_on && ns >= kSU2AosMinPasses) {
        lat_status s = su2_aos_enter(c);
        if (s != LAT_OK) return s;
        int buf = 0;
        for (int64_t k = 0; k < ns; ++k) {
            const double ck = stag == 0 ? 0.5 * h : h;
            SU2Args a = su2_args_aos(c, ck, h, buf);
            if (fixed) {   // kick at t, drift at the midpoint (reading R3)
                const double t = t0 + (double)k * h;
                su2_bg(c, a, h, scale_at(c, t), scale_at(c, t + 0.5 * h));
            }
            a.down = su2_alternate() ? (int)(k & 1) : 0;
            if ((s = su2_launch(c, kSU2StepAoS, a)) != LAT_OK) return s;
            buf ^= 1;
            stag = dir;
        }
        if ((s = su2_aos_leave(c, buf)) != LAT_OK) return s;
        c->lf_stag = dir;
        c->t = t0 + (double)ns * h;
        return LAT_OK;
    }
    for (int64_t k = 0; k < ns; ++k) {
        const double ck = stag == 0 ? 0.5 * h : h;
        const double t = t0 + (double)k * h;
        SU2Args a = fixed ? su2_args_bg(c, ck, h, scale_at(c, t), scale_at(c, t + 0.5 * h), true)
                          : su2_args(c, ck, h, true);
        a.down = su2_alternate() ? (int)(k & 1) : 0;
        lat_status s = su2_launch(c, kSU2Step, a);
        if (s != LAT_OK) return s;
        c->cur_su2 ^= 1;
        stag = dir;
    }
    c->lf_stag = dir;
    c->t = t0 + (double)ns * h;
    return LAT_OK;
}

lat_status su2_sync(lat_ctx *c)
{
    const double w = 0.5 * c->lf_stag * c->p.dt;
    if (c->p.expansion == LAT_EXP_SELF) {
        lat_status s = su2_launch(c, kSU2Energy, su2_args(c, 0.0, 0.0, false));
        if (s != LAT_OK) return s;
        U1K(u1_self_b_kick, c->sc, w, u1_self_const(c));
        U1K(u1_self_kick_w, c->sc, w, c->p.alpha);
        return su2_launch(c, kSU2Kick, su2_args_dev(c, false));
    }
    const double a = scale_at(c, c->t);
    return su2_launch(c, kSU2Kick, su2_args_bg(c, w, 0.0, a, a, false));
}

lat_status su2_energy(lat_ctx *c, lat_energies *out)
{
    const double ck = c->lf_stag != 0 ? 0.5 * c->lf_stag * c->p.dt : 0.0;
    const double V = (double)c->vol, al = c->p.alpha;
    double a = 1.0, b = 0.0;
    lat_status s;
    if (c->p.expansion == LAT_EXP_FIXED) fixed_ab(c->p, c->t, &a, &b);
    if (c->p.expansion == LAT_EXP_SELF) {
        // a and b of the record; a staggered b is half-kicked on the fly with
        // the sums of the stored half-step momenta (reading A3)
        if (ck != 0.0 && (s = su2_launch(c, kSU2Energy, su2_args(c, 0.0, 0.0, false))) != LAT_OK) return s;
        HIPCHK(c, hipMemcpyAsync(c->sc_host, c->sc, sizeof(ScaleRecord), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        a = c->sc_host->a;
        b = c->sc_host->b;
        if (ck != 0.0) {
            const double *S = c->sc_host->sums;
            const double a2 = a * a, a4 = a2 * a2, a6 = a4 * a2;
            const double Ka = std::pow(a, 2.0 * al + 1.0) / 3.0 * c->p.kappa2 *
                              ((al - 2.0) * S[0] / V / a6 + al * S[1] / V / a2 +
                               (al - 1.0) * (S[3] / V / a4 + S[4] / V / a4) + (al + 1.0) * S[2] / V);
            b += ck * Ka;
        }
    }
    s = su2_launch(c, kSU2Energy, su2_args_bg(c, ck, 0.0, a, a, false));
    if (s != LAT_OK) return s;
    HIPCHK(c, hipMemcpyAsync(c->sc_host, c->sc, sizeof(ScaleRecord), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    const double *S = c->sc_host->sums, *M = c->sc_host->maxes;
    const double a2 = a * a, a4 = a2 * a2, a6 = a4 * a2;
    out->t = c->t;
    out->a = a;
    out->b = b;
    out->EK[0] = S[0] / V / a6;
    out->EG[0] = S[1] / V / a2;
    out->EV[0] = S[2] / V;
    out->EK_B = S[3] / V / a4;
    out->EG_B = S[4] / V / a4;
    out->rho = out->EK[0] + out->EG[0] + out->EV[0] + out->EK_B + out->EG_B;
    out->hubble_lhs = b * b;
    out->hubble_rhs = std::pow(a, 2.0 * al + 2.0) * c->p.kappa2 * out->rho / 3.0;
    {
        const double den = out->hubble_lhs + out->hubble_rhs;
        out->hubble_res = den != 0.0 ? (out->hubble_lhs - out->hubble_rhs) / den : 0.0;
    }
    out->gauss_mean = S[5] / V;
    out->gauss_sum_mean = S[6] / V;
    out->gauss_abs_mean = S[7] / V;
    out->gauss_max = M[0];
    out->gauss_div_max = M[1];
    out->gauss_charge_max = M[2];
    out->step = c->step;
    return LAT_OK;
}

// Velocity-Verlet family for the U(1) and SU(2) models (a = 1): the sub-steps
// h_p = w_p h of the composition (vv_weights), one kick-and-drift
// pass per sub-step whose kick merges the half kicks that meet at its point,
// (h_{p-1} + h_p)/2, and a closing kick-only pass of h_{M-1}/2; momenta end
// at integer time.
// U(1) velocity-Verlet family with self-consistent expansion (reading R1 for
// each second-order map of the composition): kick(hs/2) at a_n, b half kick with
// E_n, a drift, field drift at the mean a, kick(hs/2) at a_{n+1}, energies,
// b half kick; every piece its own pass.
lat_status u1_step_self_vv(lat_ctx *c, int64_t ns, int dir)
{
    const double h = dir * c->p.dt;
    const std::vector<double> w = vv_weights(c->p.integrator);
    const U1SelfConst kc = u1_self_const(c);
    lat_status s;
    if ((s = u1_launch(c, kU1Energy, u1_args(c, 0.0, 0.0, false))) != LAT_OK) return s;   // E_n
    for (int64_t k = 0; k < ns; ++k)
        for (double wp : w) {
            const double hs = wp * h;
            U1K(u1_self_kick_w, c->sc, 0.5 * hs, c->p.alpha);
            if ((s = u1_launch(c, kU1Kick, u1_args_dev(c, false))) != LAT_OK) return s;
            U1K(u1_self_drift_w, c->sc, hs, 0.0, 0.5 * hs, kc, 0);
            if ((s = u1_drift_pass(c)) != LAT_OK) return s;
            u1_flip(c);
            U1K(u1_self_kick_w, c->sc, 0.5 * hs, c->p.alpha);
            if ((s = u1_kick_sums(c)) != LAT_OK) return s;
            U1K(u1_self_b_kick, c->sc, 0.5 * hs, kc);
        }
    c->t += (double)ns * h;
    return LAT_OK;
}

// SU(2) velocity-Verlet family with self-consistent expansion: as the U(1) model's.
lat_status su2_step_self_vv(lat_ctx *c, int64_t ns, int dir)
{
    const double h = dir * c->p.dt;
    const std::vector<double> w = vv_weights(c->p.integrator);
    const U1SelfConst kc = u1_self_const(c);
    lat_status s;
    if ((s = su2_launch(c, kSU2Energy, su2_args(c, 0.0, 0.0, false))) != LAT_OK) return s;   // E_n
    for (int64_t k = 0; k < ns; ++k)
        for (double wp : w) {
            const double hs = wp * h;
            U1K(u1_self_kick_w, c->sc, 0.5 * hs, c->p.alpha);
            if ((s = su2_launch(c, kSU2Kick, su2_args_dev(c, false))) != LAT_OK) return s;
            U1K(u1_self_drift_w, c->sc, hs, 0.0, 0.5 * hs, kc, 0);
            if ((s = su2_drift_pass(c)) != LAT_OK) return s;
            c->cur_su2 ^= 1;
            U1K(u1_self_kick_w, c->sc, 0.5 * hs, c->p.alpha);
            if ((s = su2_kick_sums(c)) != LAT_OK) return s;
            U1K(u1_self_b_kick, c->sc, 0.5 * hs, kc);
        }
    c->t += (double)ns * h;
    return LAT_OK;
}

lat_status gauge_step_vv(lat_ctx *c, int64_t ns, int dir)
{
    if (c->u1 && c->p.expansion == LAT_EXP_SELF) return u1_step_self_vv(c, ns, dir);
    if (c->su2 && c->p.expansion == LAT_EXP_SELF) return su2_step_self_vv(c, ns, dir);
    const double h = dir * c->p.dt;
    const std::vector<double> w = vv_weights(c->p.integrator);
    const int64_t J = (int64_t)w.size(), M = J * ns;
    const bool fixed = c->p.expansion == LAT_EXP_FIXED;
    const double t_start = c->t;
    double tk = t_start;   // time of the current kick point
    double prev = 0.0;
    const bool aos = c->su2 && c->su2_aos_on && M >= kSU2AosMinPasses;
    int buf = 0;
    if (aos) {
        lat_status s = su2_aos_enter(c);
        if (s != LAT_OK) return s;
    }
    for (int64_t p = 0; p < M; ++p) {
        const double hp = w[(size_t)(p % J)] * h;
        const double ck = 0.5 * (prev + hp);
        // fixed background: kicks at the kick point's a, drift at the
        // sub-step's midpoint (reading R3)
        if (p % J == 0) tk = t_start + (double)(p / J) * h;
        lat_status s;
        if (aos) {
            SU2Args a = su2_args_aos(c, ck, hp, buf);
            if (fixed) su2_bg(c, a, hp, scale_at(c, tk), scale_at(c, tk + 0.5 * hp));
            s = su2_launch(c, kSU2StepAoS, a);
            buf ^= 1;
        } else if (c->su2) {
            s = su2_launch(c, kSU2Step, fixed ? su2_args_bg(c, ck, hp, scale_at(c, tk), scale_at(c, tk + 0.5 * hp), true)
                                              : su2_args(c, ck, hp, true));
            c->cur_su2 ^= 1;
        } else {
            s = u1_launch(c, kU1Step, fixed ? u1_args_bg(c, ck, hp, scale_at(c, tk), scale_at(c, tk + 0.5 * hp), true)
                                            : u1_args(c, ck, hp, true));
            u1_flip(c);
        }
        tk += hp;
        if (s != LAT_OK) return s;
        prev = hp;
    }
    if (aos) {
        lat_status s = su2_aos_leave(c, buf);
        if (s != LAT_OK) return s;
    }
    const double tend = t_start + (double)ns * h;
    const double ae = scale_at(c, tend);
    lat_status s = c->su2 ? su2_launch(c, kSU2Kick, fixed ? su2_args_bg(c, 0.5 * prev, 0.0, ae, ae, false)
                                                          : su2_args(c, 0.5 * prev, 0.0, false))
                          : u1_launch(c, kU1Kick, fixed ? u1_args_bg(c, 0.5 * prev, 0.0, ae, ae, false)
                                                        : u1_args(c, 0.5 * prev, 0.0, false));
    if (s != LAT_OK) return s;
    c->t = tend;
    return LAT_OK;
}

}  // namespace

// ===========================================================================
// adjoint of the velocity-Verlet run (two fields, a = 1)
// ===========================================================================
namespace {

constexpr int kAdjTX = 64, kAdjTY = 4;

lat_status adj_pass(lat_ctx *c, double dphi, double dlam, double cA, double cB, double kL, double kV, int nb, int zc,
                    int tiles_x, int tiles_y, double *dq_slots = nullptr)
{
    AdjArgs a{};
    a.dq_slots = dq_slots;
    for (int f = 0; f < 2; ++f) {
        const int cp = c->cur_phi[f], cq = c->cur_pi[f];
        const int cl = c->cur_lam[0][f], cm = c->cur_lam[1][f];
        a.phi_in[f] = (const double *)c->phi[f][cp];
        a.pi_in[f] = (const double *)c->pi[f][cq];
        a.lphi_in[f] = (const double *)c->lam[0][f][cl];
        a.lpi_in[f] = (const double *)c->lam[1][f][cm];
        a.phi_out[f] = (double *)c->phi[f][cp ^ 1];
        a.pi_out[f] = (double *)c->pi[f][cq ^ 1];
        a.lphi_out[f] = (double *)c->lam[0][f][cl ^ 1];
        a.lpi_out[f] = (double *)c->lam[1][f][cm ^ 1];
    }
    a.N = c->N;
    a.zc = zc;
    a.tiles_x = tiles_x;
    a.tiles_y = tiles_y;
    a.inv_dx2 = 1.0 / (c->p.dx * c->p.dx);
    a.lam = c->p.lambda;
    a.q = c->p.q;
    a.dphi = dphi;
    a.dlam = dlam;
    a.cA = cA;
    a.cB = cB;
    a.kL = kL;
    a.kV = kV;
    a.partials = c->adj_partials;
    a.ticket = c->ticket;
    a.dq_acc = &c->sc->sums[kMaxQ - 1];
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    if (c->profiling) {
        lat_status st = timing_begin(c, &ev0, &ev1);
        if (st != LAT_OK) return st;
    }
    hipLaunchKernelGGL((adjoint_stage<kAdjTX, kAdjTY>), dim3(nb), dim3(kAdjTX * kAdjTY), 0, c->stream, a);
    HIPCHK(c, hipGetLastError());
    if (c->profiling) {
        lat_status st = timing_end(c, ev0, ev1, 7);
        if (st != LAT_OK) return st;
    }
    c->launches[7] += 1;
    for (int f = 0; f < 2; ++f) {
        c->cur_phi[f] ^= 1;
        c->cur_pi[f] ^= 1;
        c->cur_lam[0][f] ^= 1;
        c->cur_lam[1][f] ^= 1;
    }
    return LAT_OK;
}

lat_status checkpoint_io(lat_ctx *c, size_t j, bool store)
{
    const size_t bytes = c->vol * sizeof(double);
    for (int f = 0; f < 2; ++f) {
        double *slot_phi = c->ckpt + (j * 4 + (size_t)f) * c->vol;
        double *slot_pi = c->ckpt + (j * 4 + 2 + (size_t)f) * c->vol;
        void *phi = c->phi[f][c->cur_phi[f]], *pi = c->pi[f][c->cur_pi[f]];
        if (store) {
            HIPCHK(c, hipMemcpyAsync(slot_phi, phi, bytes, hipMemcpyDeviceToDevice, c->stream));
            HIPCHK(c, hipMemcpyAsync(slot_pi, pi, bytes, hipMemcpyDeviceToDevice, c->stream));
        } else {
            HIPCHK(c, hipMemcpyAsync(phi, slot_phi, bytes, hipMemcpyDeviceToDevice, c->stream));
            HIPCHK(c, hipMemcpyAsync(pi, slot_pi, bytes, hipMemcpyDeviceToDevice, c->stream));
        }
    }
    return LAT_OK;
}

}  // namespace

extern "C" lat_status lattice_grad(lat_ctx *c, const lat_grad_spec *spec, lat_grad_out *out)
{
    if (!c || !spec || !out) return fail(c, LAT_EINVAL, "null argument");
    c->sums_fresh = false;
    const bool spec_obs = spec->observable == LAT_OBS_SPECTRUM_BIN;
    if (spec->observable != LAT_OBS_ENERGY_FRACTION && !spec_obs)
        return fail(c, LAT_EINVAL, "unknown observable");
    if (c->batch || c->u1 || c->p.potential != LAT_PHI4_CHI2 || c->p.integrator != LAT_VV2 || c->f32)
        return fail(c, LAT_EUNSUPPORTED, "lattice_grad needs two fields, VV2 and float64");
    const bool self = c->p.expansion == LAT_EXP_SELF;
    if (spec->reserved != 0) return fail(c, LAT_EINVAL, "reserved field of lat_grad_spec must be 0");
    if (spec->field < 0 || spec->field > 1) return fail(c, LAT_EINVAL, "observable field out of range");
    if (spec_obs) {
        const long h2 = (long)(c->N / 2) * (c->N / 2);
        long bmax = (long)std::sqrt(3.0 * (double)h2);
        while ((bmax + 1) * (bmax + 1) <= 3 * h2) ++bmax;
        while (bmax * bmax > 3 * h2) --bmax;
        if (spec->bin < 1 || spec->bin > bmax) return fail(c, LAT_EINVAL, "spectrum observable: bin out of range");
    } else if (spec->bin != 0) {
        return fail(c, LAT_EINVAL, "bin is 0 for the energy fraction");
    }
    const int64_t T = spec->nsteps;
    if (T < 1 || T > (1LL << 26)) return fail(c, LAT_EINVAL, "nsteps out of range");
    if ((double)c->vol >= 4294967296.0) return fail(c, LAT_EUNSUPPORTED, "lattice_grad needs N^3 < 2^32");
    int64_t k = spec->checkpoint_stride;
    if (k <= 0) {
        k = 1;
        while (k * k < T) ++k;
    }
    if (k > T) k = T;
    const size_t ncp = (size_t)(T / k) + 1;
    const size_t bytes = c->vol * sizeof(double);
    lat_status s;

    // scratch
    for (int kk = 0; kk < 2; ++kk)
        for (int f = 0; f < 2; ++f)
            for (int b = 0; b < 2; ++b)
                if (!c->lam[kk][f][b] && hipMalloc(&c->lam[kk][f][b], bytes) != hipSuccess)
                    return fail(c, LAT_ENOMEM, "adjoint array allocation failed");
    if (ncp > c->ckpt_count) {
        if (c->ckpt) HIPCHK(c, hipFree(c->ckpt));
        c->ckpt = nullptr;
        if (hipMalloc(&c->ckpt, ncp * 4 * bytes) != hipSuccess) {
            c->ckpt_count = 0;
            return fail(c, LAT_ENOMEM, "checkpoint allocation failed");
        }
        c->ckpt_count = ncp;
    }
    const int N = c->N;
    const int tiles_x = (N + kAdjTX - 1) / kAdjTX, tiles_y = (N + kAdjTY - 1) / kAdjTY;
    int zc = (int)((long)N * tiles_x * tiles_y / 512);
    if (zc < 4) zc = 4;
    if (const char *env = std::getenv("LATTICE_ADJ_ZC")) zc = std::atoi(env);   // z chunk override
    if (zc < 1) zc = 1;
    if (zc > N) zc = N;
    const int nb = tiles_x * tiles_y * ((N + zc - 1) / zc);
    const int seed_blocks = (int)((c->vol + 255) / 256);
    const size_t need = (size_t)(nb > seed_blocks ? nb : seed_blocks) + 64;
    if (need > c->adj_partial_cap) {
        if (c->adj_partials) HIPCHK(c, hipFree(c->adj_partials));
        c->adj_partials = nullptr;
        if (hipMalloc(&c->adj_partials, need * sizeof(double)) != hipSuccess) {
            c->adj_partial_cap = 0;
            return fail(c, LAT_ENOMEM, "adjoint partials allocation failed");
        }
        c->adj_partial_cap = need;
    }
    // self-consistent reverse passes: a few sites per thread, so that every
    // block can add up all blocks' sums of the point before in its prologue
    const int rev_sites = (int)std::max<size_t>(1, (c->vol + (size_t)kSelfAdjThreads * 512 - 1) /
                                                       ((size_t)kSelfAdjThreads * 512));
    const int nbr = (int)((c->vol + (size_t)kSelfAdjThreads * rev_sites - 1) / ((size_t)kSelfAdjThreads * rev_sites));
    if (self) {
        // the k + 1 states of a segment (phi, pi of both fields) and two
        // generations of the re-run's half-step momenta
        const size_t seg_arrays = ((size_t)k + 1) * 4 + 4;
        if (seg_arrays > c->self_seg_cap) {
            if (c->self_seg) HIPCHK(c, hipFree(c->self_seg));
            c->self_seg = nullptr;
            if (hipMalloc(&c->self_seg, seg_arrays * bytes) != hipSuccess) {
                c->self_seg_cap = 0;
                return fail(c, LAT_ENOMEM, "segment state allocation failed");
            }
            c->self_seg_cap = seg_arrays;
        }
        const size_t rec_d = (sizeof(ScaleRecord) + sizeof(double) - 1) / sizeof(double);
        const size_t tneed = (size_t)2 * ((size_t)T + 1) + rec_d + 16;
        if (tneed > c->self_traj_cap) {
            if (c->self_traj) HIPCHK(c, hipFree(c->self_traj));
            c->self_traj = nullptr;
            if (hipMalloc(&c->self_traj, tneed * sizeof(double)) != hipSuccess) {
                c->self_traj_cap = 0;
                return fail(c, LAT_ENOMEM, "trajectory allocation failed");
            }
            c->self_traj_cap = tneed;
        }
        const size_t pneed = (size_t)2 * nbr * kRevQ + 3 * sizeof(SelfScalars) / sizeof(double) + 16;
        if (pneed > c->self_part_cap) {
            if (c->self_part) HIPCHK(c, hipFree(c->self_part));
            c->self_part = nullptr;
            if (hipMalloc(&c->self_part, pneed * sizeof(double)) != hipSuccess) {
                c->self_part_cap = 0;
                return fail(c, LAT_ENOMEM, "partials allocation failed");
            }
            c->self_part_cap = pneed;
        }
    }
    hipEvent_t e0, e1, e2;
    HIPCHK(c, hipEventCreate(&e0));
    HIPCHK(c, hipEventCreate(&e1));
    HIPCHK(c, hipEventCreate(&e2));
    auto cleanup = [&]() {
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        (void)hipEventDestroy(e2);
    };
#define GCHK(expr)                        \
    do {                                  \
        lat_status s_ = (expr);           \
        if (s_ != LAT_OK) {               \
            cleanup();                    \
            return s_;                    \
        }                                 \
    } while (0)

    const double h = c->p.dt, al = c->p.alpha, t_start = c->t;
    // background factors at kick point p (time t_p = t_start + p h) and of the
    // drift that leaves it: a = 1, or the fixed a(t) (kicks at t_p, drifts at
    // the midpoint)
    auto kick_l = [&](int64_t p) { return std::pow(scale_at(c, t_start + (double)p * h), 1.0 + al); };
    auto kick_v = [&](int64_t p) { return std::pow(scale_at(c, t_start + (double)p * h), 3.0 + al); };
    auto drift_d = [&](int64_t p) { return std::pow(scale_at(c, t_start + ((double)p + 0.5) * h), al - 3.0); };
    // ---- forward sweep (leapfrog form of T VV2 steps) with checkpoints
    HIPCHK(c, hipEventRecord(e0, c->stream));
    GCHK(checkpoint_io(c, 0, true));
    // self-consistent expansion: the library's own VV2 steps, one call per
    // segment between checkpoints, each pass storing (a, a') of its point on
    // the device; the scale factors come back to the host once, at the end
    // device layout of self_traj: (a, a') per step, then the initial scale record
    std::vector<double> traj_a;
    const int64_t step_save = c->step;
    double *traj_dev = c->self_traj;
    ScaleRecord *rec_dev = self ? (ScaleRecord *)(c->self_traj + 2 * ((size_t)T + 1)) : nullptr;
    if (self) {
        HIPCHK(c, hipMemcpyAsync(rec_dev, c->sc, sizeof(ScaleRecord), hipMemcpyDeviceToDevice, c->stream));
        for (int64_t s0 = 0; s0 < T; s0 += k) {
            const int64_t len = std::min<int64_t>(k, T - s0);
            c->traj_rec = traj_dev + 2 * (size_t)s0;
            const lat_status r = step_vv(c, len, 1);
            c->traj_rec = nullptr;
            GCHK(r);
            if (s0 + len < T) GCHK(checkpoint_io(c, (size_t)((s0 + len) / k), true));
        }
        std::vector<double> tr(2 * ((size_t)T + 1));
        HIPCHK(c, hipMemcpyAsync(tr.data(), traj_dev, tr.size() * sizeof(double), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        traj_a.resize((size_t)T + 1);
        for (size_t i = 0; i <= (size_t)T; ++i) traj_a[i] = tr[2 * i];
    } else {
        GCHK(reserve_coef(c, (size_t)T + 3));
        for (int64_t p = 0; p <= T; ++p) {
            PassCoef &P = c->coef_host[p];
            P.ka1 = kick_l(p);
            P.ka3 = kick_v(p);
            P.c1 = p > 0 ? 0.5 * h : 0.0;
            P.c2 = p < T ? 0.5 * h : 0.0;
            P.dend = p < T ? h * drift_d(p) : 0.0;
        }
        GCHK(upload_coef(c, (size_t)T + 1));
        for (int64_t p = 0; p < T; ++p) {
            GCHK(run_pass(c, kKickDrift, (int)p, kLastStore));
            if ((p + 1) % k == 0 && p + 1 < T) GCHK(checkpoint_io(c, (size_t)((p + 1) / k), true));
        }
        GCHK(run_pass(c, kKickOnly, (int)T, kLastStore));   // closing half kick: (phi_T, pi_T)
    }
    HIPCHK(c, hipEventRecord(e1, c->stream));

    // ---- observable and seed
    const double V = (double)c->vol;
    double O = 0.0, rho = 0.0, cb = 0.0, la_T = 0.0;
    if (spec_obs) {
        // dO/dphi_s = inverse transform of the shell-b half spectrum scaled by
        // 2 c_b; every other adjoint array starts at zero; O has no explicit q
        const int s = spec->field;
        GCHK(ensure_fft(c, false));
        GCHK(ensure_fft(c, true));
        cb = shell_weight(N, c->p.dx, spec->bin);
        hipLaunchKernelGGL(zero_doubles, dim3(1), dim3(64), 0, c->stream, &c->sc->sums[kMaxQ - 2], 2);
        HIPCHK(c, hipGetLastError());
        HIPCHK(c, hipMemcpyAsync(c->fft_in, c->phi[s][c->cur_phi[s]], bytes, hipMemcpyDeviceToDevice, c->stream));
        if (hipfftExecD2Z(c->fft_plan, c->fft_in, (hipfftDoubleComplex *)c->fft_out) != HIPFFT_SUCCESS) {
            cleanup();
            return fail(c, LAT_EHIP, "hipfftExecD2Z failed");
        }
        const size_t H = (size_t)N * N * (N / 2 + 1);
        hipLaunchKernelGGL(spectrum_shell_seed, dim3((unsigned)((H + kSpecThreads - 1) / kSpecThreads)),
                           dim3(kSpecThreads), 0, c->stream, c->fft_out, N, (long)spec->bin, 2.0 * cb,
                           c->adj_partials, c->ticket, &c->sc->sums[kMaxQ - 2]);
        HIPCHK(c, hipGetLastError());
        if (hipfftExecZ2D(c->fft_inv, (hipfftDoubleComplex *)c->fft_out, (double *)c->lam[0][s][c->cur_lam[0][s]]) !=
            HIPFFT_SUCCESS) {
            cleanup();
            return fail(c, LAT_EHIP, "hipfftExecZ2D failed");
        }
        HIPCHK(c, hipMemsetAsync(c->lam[0][1 - s][c->cur_lam[0][1 - s]], 0, bytes, c->stream));
        for (int f = 0; f < 2; ++f) HIPCHK(c, hipMemsetAsync(c->lam[1][f][c->cur_lam[1][f]], 0, bytes, c->stream));
    } else {
        GCHK(energy_sums(c, 0.0));
        const double *S = c->sc_host->sums;
        const double aT = self ? traj_a[(size_t)T] : scale_at(c, t_start + (double)T * h);
        const double ia2 = 1.0 / (aT * aT), ia6 = ia2 * ia2 * ia2;
        double EK[2], EG[2];
        for (int f = 0; f < 2; ++f) {
            EK[f] = S[f] / V / 2.0 * ia6;
            EG[f] = S[2 + f] / (c->p.dx * c->p.dx) / V / 2.0 * ia2;
        }
        rho = EK[0] + EK[1] + EG[0] + EG[1] + S[4] / V + S[5] / V;
        O = (EK[spec->field] + EG[spec->field]) / rho;
        // dO/da(T) at fixed fields: E_K ~ a^-6, E_G ~ a^-2
        const int fo = spec->field;
        const double dX = -(6.0 * EK[fo] + 2.0 * EG[fo]) / aT;
        const double drho = -(6.0 * (EK[0] + EK[1]) + 2.0 * (EG[0] + EG[1])) / aT;
        la_T = (dX - O * drho) / rho;
        hipLaunchKernelGGL(zero_doubles, dim3(1), dim3(64), 0, c->stream, &c->sc->sums[kMaxQ - 2], 2);
        HIPCHK(c, hipGetLastError());
        SeedArgs a{};
        for (int f = 0; f < 2; ++f) {
            a.phi[f] = (const double *)c->phi[f][c->cur_phi[f]];
            a.pi[f] = (const double *)c->pi[f][c->cur_pi[f]];
            a.lphi[f] = (double *)c->lam[0][f][c->cur_lam[0][f]];
            a.lpi[f] = (double *)c->lam[1][f][c->cur_lam[1][f]];
        }
        a.N = N;
        a.inv_dx2 = 1.0 / (c->p.dx * c->p.dx);
        a.lam = c->p.lambda;
        a.q = c->p.q;
        a.O = O;
        a.field = spec->field;
        a.inv_vrho = 1.0 / (V * rho);
        a.ia2 = ia2;
        a.ia6 = ia6;
        a.partials = c->adj_partials;
        a.ticket = c->ticket;
        a.out_sum = &c->sc->sums[kMaxQ - 2];
        hipLaunchKernelGGL(adjoint_seed, dim3(seed_blocks), dim3(256), 0, c->stream, a);
        HIPCHK(c, hipGetLastError());
    }

    // ---- reverse sweep
    double la = la_T, lb = 0.0, dq_self = 0.0, seed_sum = 0.0;
    if (!self) {
        // dO/dq: every block of the passes adds its partial to its own slot
        // (c->adj_partials, free once the seed has finished), summed after the
        // sweep, so no pass ends with ticket releases; LATTICE_ENERGY_DEFER=0
        // keeps the per-pass ticketed sums (the same value to rounding)
        double *slots = gauge_defer_on() ? c->adj_partials : nullptr;
        if (slots) {
            hipLaunchKernelGGL(zero_doubles, dim3((nb + 255) / 256), dim3(256), 0, c->stream, slots, nb);
            HIPCHK(c, hipGetLastError());
        }
        GCHK(adj_pass(c, 0.0, 0.0, 0.0, 0.5 * h, kick_l(T), kick_v(T), nb, zc, tiles_x, tiles_y, slots));   // closing half kick
        for (int64_t p = T - 1; p >= 0; --p) {
            const double d = h * drift_d(p);
            GCHK(adj_pass(c, -d, d, p > 0 ? 0.5 * h : 0.0, 0.5 * h, kick_l(p), kick_v(p), nb, zc, tiles_x, tiles_y,
                          slots));
            if (p % k == 0) GCHK(checkpoint_io(c, (size_t)(p / k), false));
        }
        if (slots) {
            hipLaunchKernelGGL(adj_dq_finish, dim3(1), dim3(256), 0, c->stream, (const double *)slots, nb,
                               &c->sc->sums[kMaxQ - 1]);
            HIPCHK(c, hipGetLastError());
        }
    } else {
        // Self-consistent expansion: one fused pass per time point (stage_adjoint_self.hpp),
        // the states of each segment re-run from its checkpoint with the
        // recorded scale factors; the scalar adjoints stay on the device.
        HIPCHK(c, hipMemcpyAsync(c->sc_host, c->sc, sizeof(ScaleRecord), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        seed_sum = c->sc_host->sums[kMaxQ - 2];
        const SelfConst kc{h, c->p.alpha, c->p.kappa2, V, 1.0 / (c->p.dx * c->p.dx), c->p.lambda, c->p.q};
        const double al = c->p.alpha;
        double *part[2] = {c->self_part, c->self_part + (size_t)nbr * kRevQ};
        SelfScalars *R = (SelfScalars *)(c->self_part + (size_t)2 * nbr * kRevQ);
        {
            SelfScalars s0{};
            s0.la = la_T;
            HIPCHK(c, hipMemcpyAsync(R + ((T + 1) & 1), &s0, sizeof(s0), hipMemcpyHostToDevice, c->stream));
            HIPCHK(c, hipStreamSynchronize(c->stream));
        }
        auto point = [&](int64_t n) {
            SelfPoint P{};
            P.a = traj_a[(size_t)n];
            P.ka1 = std::pow(P.a, 1.0 + al);
            P.ka3 = std::pow(P.a, 3.0 + al);
            P.pa = std::pow(P.a, al);
            P.pa2 = std::pow(P.a, 2.0 + al);
            P.C = std::pow(P.a, 2.0 * al + 1.0) / 3.0 * c->p.kappa2;
            P.kA = n < T;
            P.kB = n > 0;
            if (n > 0) {
                const double abar = 0.5 * (traj_a[(size_t)n - 1] + P.a);
                P.dr = h * std::pow(abar, al - 3.0);
                P.pbar = std::pow(abar, al - 4.0);
            }
            return P;
        };
        auto state = [&](int64_t j, int which, int f) {
            return c->self_seg + ((size_t)j * 4 + (size_t)(2 * which + f)) * c->vol;
        };
        auto carry = [&](int64_t j, int f) {
            return c->self_seg + (((size_t)k + 1) * 4 + (size_t)(2 * (j & 1) + f)) * c->vol;
        };
        const dim3 grid_site((unsigned)seed_blocks), grid_rev((unsigned)nbr), blk(kSelfAdjThreads);
        for (int64_t s0 = ((T - 1) / k) * k; s0 >= 0; s0 -= k) {
            const int64_t s1 = std::min<int64_t>(s0 + k, T);
            const int64_t m = s1 == T ? s1 - s0 : s1 - s0 - 1;   // states s0 .. s0 + m
            // re-run: the checkpoint into state 0, then m steps
            for (int64_t j = 0; j <= m; ++j) {
                SelfRerunArgs r{};
                for (int f = 0; f < 2; ++f) {
                    if (j == 0) {
                        r.phi_in[f] = c->ckpt + ((size_t)(s0 / k) * 4 + (size_t)f) * c->vol;
                        r.pp_in[f] = c->ckpt + ((size_t)(s0 / k) * 4 + 2 + (size_t)f) * c->vol;
                    } else {
                        r.phi_in[f] = state(j - 1, 0, f);
                        r.pp_in[f] = carry(j - 1, f);
                    }
                    r.phi_out[f] = state(j, 0, f);
                    r.pi_out[f] = state(j, 1, f);
                    r.pp_out[f] = carry(j, f);
                }
                const double an = traj_a[(size_t)(s0 + j)];
                r.N = N;
                r.inv_dx2 = kc.inv_dx2;
                r.lam = kc.lam;
                r.q = kc.q;
                r.ka1 = std::pow(an, 1.0 + al);
                r.ka3 = std::pow(an, 3.0 + al);
                r.ch = 0.5 * h;
                if (j > 0) {
                    r.cf = 0.5 * h;
                    r.dr = h * std::pow(0.5 * (traj_a[(size_t)(s0 + j - 1)] + an), al - 3.0);
                }
                hipLaunchKernelGGL(self_rerun, grid_site, blk, 0, c->stream, r);
                HIPCHK(c, hipGetLastError());
            }
            for (int64_t n = s0 + m; n >= s0; --n) {
                SelfRevArgs g{};
                for (int f = 0; f < 2; ++f) {
                    g.phi[f] = state(n - s0, 0, f);
                    g.pi[f] = state(n - s0, 1, f);
                    g.lphi[f] = (double *)c->lam[0][f][c->cur_lam[0][f]];
                    g.lpi_in[f] = (const double *)c->lam[1][f][c->cur_lam[1][f]];
                    g.lpi_out[f] = (double *)c->lam[1][f][c->cur_lam[1][f] ^ 1];
                }
                g.N = N;
                g.sites = rev_sites;
                g.k = kc;
                g.P = point(n);
                g.has_prev = n < T;
                if (n < T) g.Pp = point(n + 1);
                g.part_in = part[(n + 1) & 1];
                g.nb_in = nbr;
                g.part_out = part[n & 1];
                g.sc_in = R + ((n + 1) & 1);
                g.sc_out = R + (n & 1);
                hipLaunchKernelGGL(self_rev, grid_rev, blk, 0, c->stream, g);
                HIPCHK(c, hipGetLastError());
                for (int f = 0; f < 2; ++f) c->cur_lam[1][f] ^= 1;
            }
        }
        hipLaunchKernelGGL(self_rev_finish, dim3(1), blk, 0, c->stream, (const double *)part[0], nbr, point(0), kc,
                           (const SelfScalars *)R, R + 2);
        HIPCHK(c, hipGetLastError());
        {
            SelfScalars sf{};
            HIPCHK(c, hipMemcpyAsync(&sf, R + 2, sizeof(sf), hipMemcpyDeviceToHost, c->stream));
            HIPCHK(c, hipStreamSynchronize(c->stream));
            la = sf.la;
            lb = sf.lb;
            dq_self = sf.dq;
        }
        // the initial state, scale record, time and step count again
        GCHK(checkpoint_io(c, 0, false));
        HIPCHK(c, hipMemcpyAsync(c->sc, rec_dev, sizeof(ScaleRecord), hipMemcpyDeviceToDevice, c->stream));
        c->t = t_start;
        c->step = step_save;
    }
    HIPCHK(c, hipEventRecord(e2, c->stream));

    // ---- outputs
    for (int f = 0; f < 2; ++f) {
        if (out->dO_dphi[f])
            HIPCHK(c, hipMemcpyAsync(out->dO_dphi[f], c->lam[0][f][c->cur_lam[0][f]], bytes,
                                     hipMemcpyDeviceToDevice, c->stream));
        if (out->dO_dpi[f])
            HIPCHK(c, hipMemcpyAsync(out->dO_dpi[f], c->lam[1][f][c->cur_lam[1][f]], bytes,
                                     hipMemcpyDeviceToDevice, c->stream));
    }
    GCHK(settle(c));
    HIPCHK(c, hipMemcpyAsync(c->sc_host, c->sc, sizeof(ScaleRecord), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    float fms = 0.f, rms = 0.f;
    HIPCHK(c, hipEventElapsedTime(&fms, e0, e1));
    HIPCHK(c, hipEventElapsedTime(&rms, e1, e2));
    // the seed left sums[kMaxQ - 2] (shell power, or sum phi^2 chi^2 / 2); the
    // reverse sweep accumulated the coupling sensitivity in sums[kMaxQ - 1]
    // (self-consistent expansion: on the host)
    const double dq_adj = self ? dq_self : c->sc_host->sums[kMaxQ - 1];
    const double sum_seed = self ? seed_sum : c->sc_host->sums[kMaxQ - 2];
    if (spec_obs) {
        out->value = cb * sum_seed;
        out->dO_dq = dq_adj;
    } else {
        out->value = O;
        out->dO_dq = dq_adj - O * (sum_seed / V) / rho;
    }
    out->dO_da0 = self ? la : 0.0;
    out->dO_db0 = self ? lb : 0.0;
    out->forward_ms = fms;
    out->reverse_ms = rms;
    cleanup();
#undef GCHK
    return LAT_OK;
}

// ===========================================================================
// batches of independent single-field lattices
// ===========================================================================
namespace {

constexpr int kBatchTX[] = {64, 32, 16, 8, 0};   // 0: one thread per site
constexpr int kBatchSiteMaxN = 512;                // per-site mode: N^3 * 8 < 2^32

template <typename T>
BatchReal<T> make_real(lat_ctx *sub, void *scratch, int tx, int zc)
{
    BatchReal<T> R{};
    R.phi[0] = (T *)sub->phi[0][0];
    R.phi[1] = (T *)sub->phi[0][1];
    R.pi = (T *)sub->pi[0][0];
    R.pi_scratch = (T *)scratch;
    R.N = sub->N;
    if (tx == 0) {   // one thread per site
        R.tx = R.ty = R.zc = R.tiles_x = R.tiles_y = 0;
        return R;
    }
    R.tx = tx;
    R.ty = kBatchThreads / tx;
    R.zc = zc < 1 ? 1 : (zc > R.N ? R.N : zc);
    R.tiles_x = (R.N + R.tx - 1) / R.tx;
    R.tiles_y = (R.N + R.ty - 1) / R.ty;
    return R;
}

int real_blocks(int N, int tx, int zc)
{
    if (tx == 0) return (int)(((size_t)N * N * N + kBatchThreads - 1) / kBatchThreads);
    const int ty = kBatchThreads / tx;
    return ((N + tx - 1) / tx) * ((N + ty - 1) / ty) * ((N + zc - 1) / zc);
}

constexpr int kXcds = 8;

// realization descriptors with the tiles in c->batch_tile
template <typename T>
std::vector<BatchReal<T>> batch_reals(lat_ctx *c)
{
    const int n = (int)c->subs.size();
    std::vector<BatchReal<T>> reals(n);
    for (int r = 0; r < n; ++r) {
        const auto tz = c->batch_tile[c->subs[r]->N];
        reals[r] = make_real<T>(c->subs[r], c->pi_scratch[r], tz.first, tz.second);
    }
    return reals;
}

// Block table for the realizations in `list`, in dispatch order.  Blocks are
// dispatched round-robin over the 8 XCDs (block b on XCD b % 8), so the table
// is built per XCD and interleaved: whole realizations go to the XCD with the
// fewest sites so far (largest first), each XCD's list starts with its longest
// blocks (z-marching tiles by chunk length, then one-site blocks), and shorter
// lists are padded with empty entries.
template <typename T>
std::vector<int2> make_block_table(const std::vector<BatchReal<T>> &reals, std::vector<int> list)
{
    std::stable_sort(list.begin(), list.end(), [&](int a, int b) { return reals[a].N > reals[b].N; });
    std::vector<std::vector<int>> per(kXcds);
    std::vector<double> load(kXcds, 0.0);
    for (int r : list) {
        const int x = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        per[x].push_back(r);
        load[x] += (double)reals[r].N * reals[r].N * reals[r].N;
    }
    std::vector<std::vector<int2>> seq(kXcds);
    size_t longest = 0;
    for (int x = 0; x < kXcds; ++x) {
        std::stable_sort(per[x].begin(), per[x].end(), [&](int a, int b) {
            const int wa = reals[a].tx ? reals[a].zc : 0, wb = reals[b].tx ? reals[b].zc : 0;
            return wa > wb;
        });
        for (int r : per[x]) {
            const int nb = real_blocks(reals[r].N, reals[r].tx, reals[r].zc);
            for (int b = 0; b < nb; ++b) seq[x].push_back(make_int2(r, b));
        }
        longest = std::max(longest, seq[x].size());
    }
    std::vector<int2> blocks(longest * kXcds, make_int2(-1, 0));
    for (int x = 0; x < kXcds; ++x)
        for (size_t j = 0; j < seq[x].size(); ++j) blocks[j * kXcds + x] = seq[x][j];
    return blocks;
}

// Upload the realization table and the block table for the realizations in
// `which` (all when empty); the launch without a segment uses it.
template <typename T>
lat_status build_tables(lat_ctx *c, const std::vector<int> &which)
{
    const int n = (int)c->subs.size();
    const std::vector<BatchReal<T>> reals = batch_reals<T>(c);
    std::vector<int> list = which;
    if (list.empty())
        for (int r = 0; r < n; ++r) list.push_back(r);
    const std::vector<int2> blocks = make_block_table<T>(reals, list);
    const size_t rbytes = (size_t)n * sizeof(BatchReal<T>);
    if (!c->reals_dev && hipMalloc(&c->reals_dev, rbytes) != hipSuccess)
        return fail(c, LAT_ENOMEM, "batch table allocation failed");
    if ((int)blocks.size() > c->batch_blocks) {
        if (c->block_work) HIPCHK(c, hipFree(c->block_work));
        c->block_work = nullptr;
        if (hipMalloc(&c->block_work, blocks.size() * sizeof(int2)) != hipSuccess)
            return fail(c, LAT_ENOMEM, "batch block table allocation failed");
        c->batch_blocks = (int)blocks.size();
    }
    HIPCHK(c, hipMemcpy(c->reals_dev, reals.data(), rbytes, hipMemcpyHostToDevice));
    HIPCHK(c, hipMemcpy(c->block_work, blocks.data(), blocks.size() * sizeof(int2), hipMemcpyHostToDevice));
    c->reals_host.assign((const char *)reals.data(), (const char *)reals.data() + rbytes);
    c->nblocks = (int)blocks.size();
    return LAT_OK;
}

// Step segments: realizations (largest first) grouped so that each group's
// working set (phi in both buffers and pi) stays under a byte budget sized for
// the 256 MB Infinity Cache; lattice_step runs all its steps on one segment
// before the next, so a segment's arrays stay cache-resident across steps.
// The realizations are independent, so the order changes no result.
constexpr double kSegBudgetMB = 128.0;

template <typename T>
lat_status build_segments(lat_ctx *c)
{
    for (int2 *t : c->seg_work) (void)hipFree(t);
    c->seg_work.clear();
    c->seg_blocks.clear();
    double budget = kSegBudgetMB;
    if (const char *env = std::getenv("LATTICE_BATCH_SEG_MB")) budget = std::atof(env);
    if (!(budget > 0.0)) return LAT_OK;   // one launch over all realizations per step
    const int n = (int)c->subs.size();
    const std::vector<BatchReal<T>> reals = batch_reals<T>(c);
    std::vector<int> order(n);
    for (int r = 0; r < n; ++r) order[r] = r;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return reals[a].N > reals[b].N; });
    std::vector<std::vector<int>> segs(1);
    double bytes = 0.0;
    for (int r : order) {
        const double rb = 3.0 * (double)c->subs[r]->vol * c->esize;
        if (!segs.back().empty() && bytes + rb > budget * 1048576.0) {
            segs.emplace_back();
            bytes = 0.0;
        }
        segs.back().push_back(r);
        bytes += rb;
    }
    if (segs.size() < 2) return LAT_OK;
    for (const auto &sg : segs) {
        const std::vector<int2> blocks = make_block_table<T>(reals, sg);
        int2 *d = nullptr;
        if (hipMalloc(&d, blocks.size() * sizeof(int2)) != hipSuccess)
            return fail(c, LAT_ENOMEM, "batch segment table allocation failed");
        c->seg_work.push_back(d);
        c->seg_blocks.push_back((int)blocks.size());
        HIPCHK(c, hipMemcpy(d, blocks.data(), blocks.size() * sizeof(int2), hipMemcpyHostToDevice));
    }
    c->graph_n = 0;
    return LAT_OK;
}

template <typename T>
BatchArgs<T> batch_args(lat_ctx *c, int pass_index, int parity, int tuning)
{
    BatchArgs<T> a{};
    a.reals = (const BatchReal<T> *)c->reals_dev;
    a.block_work = c->block_work;
    a.coef = c->coef + pass_index;
    a.parity = parity;
    a.tuning = tuning;
    a.inv_dx2 = 1.0 / (c->p.dx * c->p.dx);
    a.lam = c->p.lambda;
    return a;
}

template <typename T>
lat_status batch_launch(lat_ctx *c, hipStream_t s, int pass_index, int parity, int tuning, int seg = -1)
{
    BatchArgs<T> a = batch_args<T>(c, pass_index, parity, tuning);
    int nb = c->nblocks;
    if (seg >= 0) {
        a.block_work = c->seg_work[seg];
        nb = c->seg_blocks[seg];
    }
    hipLaunchKernelGGL(batch_lf_stage<T>, dim3(nb), dim3(kBatchThreads), 0, s, a);
    HIPCHK(c, hipGetLastError());
    return LAT_OK;
}

// Autotuner: per lattice size, time the candidate tile widths and z chunks on
// the realizations of that size (writing only to shadow / scratch buffers).
template <typename T>
lat_status autotune(lat_ctx *c)
{
    std::map<int, std::vector<int>> groups;
    for (int r = 0; r < (int)c->subs.size(); ++r) groups[c->subs[r]->N].push_back(r);
    lat_status s = reserve_coef(c, 2);
    if (s != LAT_OK) return s;
    c->coef_host[0].ka1 = c->coef_host[0].ka3 = 1.0;
    c->coef_host[0].c1 = 0.5 * c->p.dt;
    c->coef_host[0].dend = c->p.dt;
    if ((s = upload_coef(c, 1)) != LAT_OK) return s;
    hipEvent_t e0, e1;
    HIPCHK(c, hipEventCreate(&e0));
    HIPCHK(c, hipEventCreate(&e1));
    for (auto &g : groups) {
        const int N = g.first;
        float best = 1e30f;
        std::pair<int, int> best_cfg = c->batch_tile[N];
        for (int tx : kBatchTX) {
            if (tx > 2 * N && tx != 8) continue;
            const int zcs[] = {4, 8, 16, 32, N};
            for (int zc : zcs) {
                // one candidate for the per-site mode, which forms 32-bit byte offsets
                if (zc > N || (tx == 0 && (zc != 4 || N > kBatchSiteMaxN))) continue;
                c->batch_tile[N] = {tx, zc};
                if ((s = build_tables<T>(c, g.second)) != LAT_OK) return s;
                if ((s = batch_launch<T>(c, c->stream, 0, 0, 1)) != LAT_OK) return s;   // warm
                HIPCHK(c, hipEventRecord(e0, c->stream));
                for (int it = 0; it < 3; ++it)
                    if ((s = batch_launch<T>(c, c->stream, 0, 0, 1)) != LAT_OK) return s;
                HIPCHK(c, hipEventRecord(e1, c->stream));
                HIPCHK(c, hipEventSynchronize(e1));
                float ms = 0.f;
                HIPCHK(c, hipEventElapsedTime(&ms, e0, e1));
                if (ms < best) {
                    best = ms;
                    best_cfg = {tx, zc};
                }
            }
        }
        c->batch_tile[N] = best_cfg;
    }
    // refine: with every realization stepped as lattice_step runs them (one
    // launch over all, or segment after segment, sharing the caches and the
    // XCDs), revisit each size's shape, largest size first
    if (groups.size() > 1) {
        auto time_all = [&](float *ms) -> lat_status {
            lat_status st = build_tables<T>(c, {});
            if (st != LAT_OK) return st;
            if ((st = build_segments<T>(c)) != LAT_OK) return st;
            const int nseg = c->seg_work.empty() ? 1 : (int)c->seg_work.size();
            auto pass = [&](int reps) -> lat_status {
                for (int g = 0; g < nseg; ++g)
                    for (int it = 0; it < reps; ++it) {
                        lat_status r = batch_launch<T>(c, c->stream, 0, 0, 1, c->seg_work.empty() ? -1 : g);
                        if (r != LAT_OK) return r;
                    }
                return LAT_OK;
            };
            if ((st = pass(1)) != LAT_OK) return st;   // warm
            HIPCHK(c, hipEventRecord(e0, c->stream));
            if ((st = pass(3)) != LAT_OK) return st;
            HIPCHK(c, hipEventRecord(e1, c->stream));
            HIPCHK(c, hipEventSynchronize(e1));
            HIPCHK(c, hipEventElapsedTime(ms, e0, e1));
            return LAT_OK;
        };
        for (auto g = groups.rbegin(); g != groups.rend(); ++g) {
            const int N = g->first;
            float best = 0.f;
            if ((s = time_all(&best)) != LAT_OK) return s;
            std::pair<int, int> best_cfg = c->batch_tile[N];
            for (int tx : kBatchTX) {
                if (tx > 2 * N && tx != 8) continue;
                const int zcs[] = {4, 8, 16, 32, N};
                for (int zc : zcs) {
                    if (zc > N || (tx == 0 && (zc != 4 || N > kBatchSiteMaxN))) continue;
                    c->batch_tile[N] = {tx, zc};
                    float ms = 0.f;
                    if ((s = time_all(&ms)) != LAT_OK) return s;
                    if (ms < best) {
                        best = ms;
                        best_cfg = {tx, zc};
                    }
                }
            }
            c->batch_tile[N] = best_cfg;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return LAT_OK;
}

template <typename T>
lat_status batch_step_t(lat_ctx *c, int64_t ns)
{
    const double h = c->p.dt, al = c->p.alpha;
    lat_status s = reserve_coef(c, (size_t)ns + 1);
    if (s != LAT_OK) return s;
    const double t_start = c->t;
    int stag = c->lf_stag;
    for (int64_t k = 0; k < ns; ++k) {
        PassCoef &P = c->coef_host[k];
        const double t = t_start + (double)k * h;
        const double a = scale_at(c, t);
        P.ka1 = std::pow(a, 1.0 + al);
        P.ka3 = std::pow(a, 3.0 + al);
        P.c1 = stag == 0 ? 0.5 * h : h;
        P.dend = h * std::pow(scale_at(c, t + 0.5 * h), al - 3.0);
        P.t = t;
        stag = 1;
    }
    if ((s = upload_coef(c, (size_t)ns)) != LAT_OK) return s;
    const bool eager = std::getenv("LATTICE_NO_GRAPH") != nullptr;
    // all steps of one segment, then the next (a single segment: every realization per launch)
    const int nseg = c->seg_work.empty() ? 1 : (int)c->seg_work.size();
    auto enqueue = [&](hipStream_t st) -> lat_status {
        for (int g = 0; g < nseg; ++g)
            for (int64_t k = 0; k < ns; ++k) {
                lat_status r = batch_launch<T>(c, st, (int)k, (int)((c->batch_parity + k) & 1), 0,
                                               c->seg_work.empty() ? -1 : g);
                if (r != LAT_OK) return r;
            }
        return LAT_OK;
    };
    if (eager && (s = enqueue(c->stream)) != LAT_OK) return s;
    // (re)capture the graph of ns batched passes starting at the current parity
    if (!eager && (!c->graph_exec || c->graph_n != ns || c->graph_parity != c->batch_parity)) {
        if (c->graph_exec) HIPCHK(c, hipGraphExecDestroy(c->graph_exec));
        if (c->graph) HIPCHK(c, hipGraphDestroy(c->graph));
        c->graph_exec = nullptr;
        c->graph = nullptr;
        HIPCHK(c, hipStreamBeginCapture(c->capture_stream, hipStreamCaptureModeThreadLocal));
        s = enqueue(c->capture_stream);
        if (s != LAT_OK) {
            hipGraph_t g = nullptr;
            (void)hipStreamEndCapture(c->capture_stream, &g);
            if (g) (void)hipGraphDestroy(g);
            return s;
        }
        HIPCHK(c, hipStreamEndCapture(c->capture_stream, &c->graph));
        HIPCHK(c, hipGraphInstantiate(&c->graph_exec, c->graph, nullptr, nullptr, 0));
        c->graph_n = ns;
        c->graph_parity = c->batch_parity;
    }
    if (!eager) HIPCHK(c, hipGraphLaunch(c->graph_exec, c->stream));
    c->launches[4] += ns * nseg;
    c->batch_parity = (int)((c->batch_parity + ns) & 1);
    if (c->batch_parity == 1) {
        const int n = (int)c->subs.size();
        hipLaunchKernelGGL(batch_settle<T>, dim3(64, n), dim3(256), 0, c->stream,
                           (const BatchReal<T> *)c->reals_dev, n, 1);
        HIPCHK(c, hipGetLastError());
        c->batch_parity = 0;
    }
    c->t = t_start + (double)ns * h;
    c->lf_stag = 1;
    for (lat_ctx *sub : c->subs) {
        sub->t = c->t;
        sub->lf_stag = 1;
        sub->step += ns;
    }
    return LAT_OK;
}

lat_status batch_step(lat_ctx *c, int64_t nsteps)
{
    if (nsteps < 0) return fail(c, LAT_EUNSUPPORTED, "batch contexts step forward only");
    lat_status s = c->f32 ? batch_step_t<float>(c, nsteps) : batch_step_t<double>(c, nsteps);
    if (s == LAT_OK) c->step += nsteps;
    return s;
}

}  // namespace

extern "C" lat_status lattice_init_batch(lat_ctx **out, const lat_params *p, int32_t n_real,
                                         const int32_t *N_per_real, const lat_fields *f, int32_t tune,
                                         void *stream)
{
    if (!out) return fail(nullptr, LAT_EINVAL, "null ctx pointer");
    *out = nullptr;
    if (!p || !N_per_real || !f || n_real < 1 || n_real > (1 << 20))
        return fail(nullptr, LAT_EINVAL, "bad batch arguments");
    if (p->potential != LAT_PHI4 || p->integrator != LAT_LF ||
        (p->expansion != LAT_EXP_NONE && p->expansion != LAT_EXP_FIXED))
        return fail(nullptr, LAT_EUNSUPPORTED, "batches are provided for one field, LF, no or fixed expansion");
    // every realization's parameters and pointers are checked before anything is allocated
    for (int r = 0; r < n_real; ++r) {
        lat_params pr = *p;
        pr.N = N_per_real[r];
        const lat_status vs = validate(&pr, &f[r]);
        if (vs != LAT_OK) {
            g_init_error = "realization " + std::to_string(r) + ": " + g_init_error;
            return vs;
        }
    }
    lat_ctx *c = new (std::nothrow) lat_ctx();
    if (!c) return fail(nullptr, LAT_ENOMEM, "host allocation failed");
    c->p = *p;
    c->batch = true;
    c->stream = (hipStream_t)stream;
    c->f32 = p->precision == LAT_PREC_F32;
    c->esize = c->f32 ? 4 : 8;
    c->nf = 1;
    c->t = p->t0;
    c->lf_stag = p->lf_staggered;
    auto bail = [&](lat_status st, const std::string &m) {
        free_ctx(c);
        g_init_error = m;
        return st;
    };
    for (int r = 0; r < n_real; ++r) {
        lat_params pr = *p;
        pr.N = N_per_real[r];
        lat_ctx *sub = nullptr;
        lat_status st = lattice_init(&sub, &pr, &f[r], stream);
        if (st != LAT_OK) return bail(st, "realization " + std::to_string(r) + ": " + g_init_error);
        c->subs.push_back(sub);
        void *scr = nullptr;
        if (hipMalloc(&scr, sub->vol * c->esize) != hipSuccess) return bail(LAT_ENOMEM, "scratch allocation failed");
        c->pi_scratch.push_back(scr);
        c->vol += sub->vol;
        if (!c->batch_tile.count(sub->N)) {
            const int N = sub->N;
            const int tx = N % 64 == 0 ? 64 : N % 32 == 0 ? 32 : N % 16 == 0 ? 16 : 8;
            c->batch_tile[N] = {tx, N >= 48 ? 16 : 8};
            // LATTICE_BATCH_TILE="tx,zc" (tx in {64, 32, 16, 8}) or "site" sets the
            // shape of every size when the autotuner is off
            if (const char *env = std::getenv("LATTICE_BATCH_TILE")) {
                int etx = 0, ezc = 0;
                if (std::strcmp(env, "site") == 0 && N <= kBatchSiteMaxN) c->batch_tile[N] = {0, 0};
                else if (std::sscanf(env, "%d,%d", &etx, &ezc) == 2 && (etx == 64 || etx == 32 || etx == 16 ||
                                                                        etx == 8) && ezc >= 1)
                    c->batch_tile[N] = {etx, ezc};
            }
        }
    }
    if (hipStreamCreateWithFlags(&c->capture_stream, hipStreamNonBlocking) != hipSuccess)
        return bail(LAT_EHIP, "stream creation failed");
    for (auto &e : c->ring_ev)
        if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess)
            return bail(LAT_EHIP, "event creation failed");
    if (hipStreamSynchronize(c->stream) != hipSuccess) return bail(LAT_EHIP, "stream synchronize failed");
    lat_status st;
    if (tune) {
        st = c->f32 ? autotune<float>(c) : autotune<double>(c);
        if (st != LAT_OK) return bail(st, c->err);
    }
    st = c->f32 ? build_tables<float>(c, {}) : build_tables<double>(c, {});
    if (st != LAT_OK) return bail(st, c->err);
    st = c->f32 ? build_segments<float>(c) : build_segments<double>(c);
    if (st != LAT_OK) return bail(st, c->err);
    if (hipStreamSynchronize(c->stream) != hipSuccess) return bail(LAT_EHIP, "stream synchronize failed");
    *out = c;
    return LAT_OK;
}

extern "C" lat_status lattice_energy_batch(lat_ctx *c, int32_t r, lat_energies *out)
{
    if (!c || !out) return fail(c, LAT_EINVAL, "null argument");
    if (!c->batch || r < 0 || r >= (int)c->subs.size()) return fail(c, LAT_EINVAL, "bad realization index");
    lat_status s = lattice_energy(c->subs[r], out);
    if (s != LAT_OK) return fail(c, s, c->subs[r]->err);
    return LAT_OK;
}

extern "C" lat_status lattice_batch_tile(const lat_ctx *c, int32_t N, int32_t *tx, int32_t *ty, int32_t *zc)
{
    if (!c || !c->batch || !tx || !ty || !zc) return LAT_EINVAL;
    auto it = c->batch_tile.find(N);
    if (it == c->batch_tile.end()) return LAT_EINVAL;
    *tx = it->second.first;
    *ty = it->second.first ? kBatchThreads / it->second.first : 0;
    *zc = it->second.first ? it->second.second : 0;
    return LAT_OK;
}
