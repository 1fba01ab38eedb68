// Internal declarations shared by the kernels (lb_kernels.hip) and the host
// side of the C ABI (lb_api.hip). Nothing here is visible to callers of lb.h.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbm {

// ---------------------------------------------------------------------------
// Device-memory layout of one lattice ("arena", one allocation):
//   buf[0], buf[1]  population buffers (A/B ping-pong; one buffer, buf[1] ==
//                   buf[0], when updated in place), row-interleaved: row y
//                   is one block of row_bytes holding, one after another, the
//                   pitch-long rows (pitch = nx rounded up to 64) of the 18
//                   planes f_0..f_8, g_0..g_8. In the 16-bit formats a block
//                   holds 32-bit words pairing f_i and g_i for i = 2, 4..8 (f in
//                   the low half), the 16-bit rows of g_1 and g_3, then 32-bit
//                   rows of f_1, f_3, f_0 and g_0 (g_0 at byte g0_offset). Every
//                   format except FP64 stores f_i - r_i, r_i the rest state at
//                   rho_ref in a bulk phase, and g_0 split as b + q (G0Code in
//                   the kernels).
//   band            (in place only) pitch*ny 8-byte words: phi of S_n at the
//                   nodes along tile borders, written by the pre-pass of each
//                   step (FP64 or FP32 values); between steps, scratch space.
//   nbr             pitch*ny bytes. 0xFF marks a solid node; for a fluid node
//                   bit (i-1) is set when the pull source r - e_i is solid.
//   grec            pitch*ny bytes, used at solid nodes: bits 0..3 mark fluid
//                   axis neighbours s + e_1..e_4, bits 4..7 fluid diagonal
//                   neighbours s + e_5..e_8.
//   dphi            pitch*ny wall gradients d_perp phi (FP64 for the FP64
//                   format, FP32 otherwise), read at solid nodes.
//   misc            per-workgroup FP64 partial sums, the last diagnostics,
//                   the sticky numeric-error flag, the crossing counter and
//                   this lattice's View and tile table.
// buf[1] also serves as staging space for initial fields, read-back fields and
// contact-line crossings between steps (it is rewritten in full by every step);
// in place, the band plane does (and the node's own slots stage rho0, u0).
//
// In-place update (two phases). Phase 0 reads the layout "X", in which the
// post-collision f_i of node r sits at r in plane OPP(i): the pull takes f_i
// from r - e_i in plane OPP(i) (or, across a solid link, from r in plane i),
// and the node writes its f'_i to r + e_i in plane i (or, toward a solid
// neighbour, to r in plane OPP(i)), which is the layout "P": the populations
// arriving at r sit at r in plane i. Phase 1 reads P at r and writes f'_i to r
// in plane OPP(i), layout X again. In both phases the slots a node writes are
// the slots it read, and no two fluid nodes share a slot. S_0 is written in
// layout P, so step n runs phase (n + 1) mod 2.
// ---------------------------------------------------------------------------

enum Storage { ST_F64 = 0, ST_F32 = 1, ST_F16S = 2, ST_BF16S = 3, ST_F64C = 4, ST_F32C = 5 };
enum Collision { CO_BGK = 0, CO_MRT = 1 };

constexpr int kPitchAlign = 64;     // elements
constexpr int kNR = 8;              // rows of the phi ring buffer in LDS
constexpr int kPartials = 8;        // doubles per workgroup partial record

struct View {
    int32_t nx, ny, pitch, tiles_x;
    int64_t plane;            // nodes per plane including row padding (pitch * ny)
    int64_t row_bytes;        // bytes of one row block of a population buffer
    int64_t g0_offset;        // byte offset of the 32-bit g_0 row inside a block (16-bit;
                              // the 32-bit f_1, f_3, f_0 rows precede it)
    char* buf[2];
    void* band;               // in place: phi of the tile-border nodes of S_n
    const uint8_t* nbr;
    const uint8_t* grec;
    const void* dphi;
    double A, B, kappa, Gamma, tau_alpha, tau_beta, inv_tau_phi;
    double rho_ref, p0_ref;   // rest state of the shifted formats: f_i - r_i is stored
    int32_t zero_u_feq, zero_u_geq;
    int32_t storage, collision;
    int32_t tau_clamp, inplace;
    int32_t tau_lut, bounce;  // tau table size (0 = Eq. (tau)); lattice-node bounce-back
    double tau_step;          // (tau_alpha - tau_beta) / (tau_lut - 1)
};

struct Tile {
    int32_t member, tx, ty;  // member -1: an empty entry (padding of a batch's stepwise table)
    int32_t id;      // logical tile index (member-major, row-major): its partial-sum record
    int32_t y0, y1;  // rows y0 .. y1-1 of the member (strip heights may differ per member)
};

// XCD-aware order of workgroups: the device hands consecutive workgroup ids to
// its 8 XCDs in turn, so workgroup b runs on XCD b % 8. Workgroup b is given
// logical tile xcd_tile(b, n): each XCD receives one contiguous range of tiles
// (row-major), so neighbouring tiles, which share halo cache lines, run at the
// same time on the same XCD and share its L2.
__host__ __device__ inline int xcd_tile(int b, int n) {
    const int g = b & 7, k = b >> 3, q = n >> 3, r = n & 7;
    return g * q + (g < r ? g : r) + k;
}

// Offsets of one lattice inside its arena.
struct Layout {
    int32_t pitch;
    int64_t plane;
    size_t row_bytes;       // bytes of one row block of a population buffer
    size_t buf_bytes;       // bytes of one population buffer
    size_t g0_offset;
    size_t off_buf0, off_buf1, off_band, off_nbr, off_grec, off_dphi, off_misc;
    size_t n_partials;      // partial records available
    size_t off_partials, off_diag, off_flag, off_counter, off_view, off_tiles;
    size_t n_tiles_max;
    size_t total;
};

Layout make_layout(int nx, int ny, int storage, bool inplace);

// Kernel launchers (lb_kernels.hip). All enqueue on `stream` and return the
// hipError_t of the launch.
hipError_t launch_sweep(int storage, int collision, int block_x, bool diag, bool tau_phi_one,
                        bool inplace, const View* d_views, const Tile* d_tiles, int n_blocks_1d,
                        int grid_x, int grid_y, int rows, int parity, double* partials,
                        hipStream_t stream);
// Persistent window of `steps` timesteps of a batch (sweep_persistent_kernel):
// `grid` workgroups claim (step, tile) items from *next in step-major order and
// wait on done[] for the tiles listed in d_deps (kPersistDeps per tile, -1 =
// none). done[] and *next must be zero at the start; *err is set when a wait
// exceeds spin_limit polls. block_x 128, 256 or 512; no periodic check.
constexpr int kPersistDeps = 16;
hipError_t launch_persistent(int storage, int collision, int block_x, bool tau_phi_one,
                             const View* d_views, const Tile* d_tiles, const int32_t* d_deps,
                             int n_tiles, int steps, int parity0, int grid, int32_t* done,
                             uint32_t* next, int32_t* err, uint32_t spin_limit,
                             hipStream_t stream);
hipError_t persistent_occupancy(int storage, int collision, int block_x, bool tau_phi_one,
                                int* per_cu);
// Lattice-node bounce-back: the wall nodes' reversal for one step, over the
// same tiles as the sweep (members whose bounce is 0 are skipped).
hipError_t launch_walls(int storage, int block_x, const View* d_views, const Tile* d_tiles,
                        int n_blocks_1d, int grid_x, int grid_y, int rows, int parity,
                        hipStream_t stream);
// In place: phi of S_n at the nodes of the two rows and columns along every
// tile border of the (block_x, rows) tiling, into View::band.
hipError_t launch_band(int storage, bool tau_phi_one, const View* d_view, int nx, int ny,
                       int block_x, int rows, int parity, hipStream_t stream);
hipError_t launch_finalize(const Tile* d_tiles, const int32_t* member_first, int n_members,
                           int n_records_single, const double* partials, double* diag_out,
                           int32_t* flag, hipStream_t stream);
hipError_t launch_init_state(const View& v, const double* phi0, const double* rho0,
                             const double* ux0, const double* uy0, hipStream_t stream);
hipError_t launch_moments(const View& v, int parity, int64_t first, int64_t count,
                          double* fields, double* partials, int n_records, int32_t x_lo,
                          int32_t x_hi, hipStream_t stream);
hipError_t launch_read_plane(const View& v, int parity, int plane, double* out,
                             hipStream_t stream);
hipError_t launch_crossings(const View& v, int parity, void* points, int64_t capacity,
                            unsigned long long* counter, hipStream_t stream);
hipError_t launch_fill(void* dst, uint8_t value, size_t bytes, hipStream_t stream);
hipError_t launch_stream_copy(const void* src, void* dst, size_t bytes, int blocks, int variant,
                              hipStream_t stream);

struct Crossing {
    uint64_t key;   // (node << 2) | (axis << 1) | (phi > 0 at the base node)
    double t;       // fraction along the link from the base node
};

}  // namespace lbm
