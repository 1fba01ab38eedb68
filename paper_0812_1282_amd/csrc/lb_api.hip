// Host side of the C ABI declared in include/lb.h.
//
// A "group" holds one or more lattices ("members") that advance together:
// lb_handle is a group of one, lb_batch a group of n. Each member owns an
// arena (see lb_internal.h) inside the group's device allocation; a batched
// step is one launch over the tiles of every member.
#include "lb.h"
#include "lb_internal.h"

#include <hip/hip_runtime.h>
#include <rocprofiler-sdk-roctx/roctx.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

using namespace lbm;

namespace {

thread_local std::string g_err = "no error";

int fail(int code, const std::string& msg) {
    g_err = msg;
    return code;
}

// A host-side roctx range for the lifetime of a scope: a profiler run with
// marker tracing shows each entry point, graph capture and graph replay on the
// host timeline; without a profiler the calls return at once.
struct Range {
    explicit Range(const char* name) { roctxRangePushA(name); }
    ~Range() { roctxRangePop(); }
    Range(const Range&) = delete;
    Range& operator=(const Range&) = delete;
};

#define HIPCHK(call)                                                                       \
    do {                                                                                   \
        hipError_t e_ = (call);                                                            \
        if (e_ != hipSuccess)                                                              \
            return fail(LB_EHIP, std::string(#call) + ": " + hipGetErrorString(e_));       \
    } while (0)

constexpr int kEX[9] = {0, 1, -1, 0, 0, 1, -1, -1, 1};
constexpr int kEY[9] = {0, 0, 0, 1, -1, 1, -1, 1, -1};
constexpr int kGraphSteps = 32;  // longest window of timesteps in one captured graph
constexpr int kGraphLens = 6;    // windows of 1, 2, 4, ..., 32 steps
constexpr int kBatchTuneSteps = 4;  // timed steps per candidate when lb_batch_init tunes
constexpr uint32_t kDefaultSpinLimit = 1u << 20;  // polls before a persistent wait gives up

size_t round_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

}  // namespace

namespace lbm {

Layout make_layout(int nx, int ny, int storage, bool inplace) {
    Layout L{};
    L.pitch = (int32_t)round_up((size_t)nx, kPitchAlign);
    L.plane = (int64_t)L.pitch * ny;
    const size_t plane = (size_t)L.plane;
    const size_t pitch = (size_t)L.pitch;
    if (storage == ST_F64) {
        L.row_bytes = 18 * pitch * 8;
    } else if (storage == ST_F32) {
        L.row_bytes = 18 * pitch * 4;
    } else if (storage == ST_F64C) {
        L.row_bytes = 13 * pitch * 8;  // f_0..f_8, then phi, Gamma mu, u_x, u_y
    } else if (storage == ST_F32C) {
        L.row_bytes = 13 * pitch * 4;
    } else {
        // f_2, f_4..f_8, g_1..g_8 in 16 bits, then f_1, f_3, f_0, g_0 in 32 bits
        L.g0_offset = 14 * pitch * 2 + 3 * pitch * 4;
        L.row_bytes = L.g0_offset + pitch * 4;
    }
    L.buf_bytes = round_up(L.row_bytes * ny, 256);
    const size_t dsz = (storage == ST_F64 || storage == ST_F64C) ? 8 : 4;
    L.off_buf0 = 0;
    if (inplace) {  // one population buffer, then the band plane (8 bytes per node)
        L.off_buf1 = 0;
        L.off_band = L.buf_bytes;
        L.off_nbr = L.off_band + round_up(plane * 8, 256);
    } else {
        L.off_buf1 = L.buf_bytes;
        L.off_band = 0;
        L.off_nbr = 2 * L.buf_bytes;
    }
    L.off_grec = L.off_nbr + round_up(plane, 256);
    L.off_dphi = L.off_grec + round_up(plane, 256);
    L.off_misc = L.off_dphi + round_up(plane * dsz, 256);
    const size_t tiles_max = ((size_t)(nx + 63) / 64) * (size_t)ny;
    const size_t node_blocks = ((size_t)nx * ny + 255) / 256;
    L.n_partials = std::max(tiles_max, node_blocks) + 1;
    L.n_tiles_max = tiles_max;
    L.off_partials = L.off_misc;
    L.off_diag = L.off_partials + round_up(L.n_partials * kPartials * 8, 256);
    L.off_flag = L.off_diag + 256;
    L.off_counter = L.off_flag + 256;
    L.off_view = L.off_counter + 256;
    L.off_tiles = L.off_view + round_up(sizeof(View), 256);
    L.total = L.off_tiles;
    return L;
}

}  // namespace lbm

// Scratch of lb_diagnostics_noalloc: the per-block partial records of the
// moments reduction, the finished record and a flag word, in a file-scope device
// array instead of the lattice's arena, so that the call allocates nothing.
// Every GPU the library runs on holds its own copy until the process ends.
constexpr size_t kScratchRecords = (size_t)1 << 15;  // one per 256 nodes: up to 2^23 nodes
constexpr size_t kScratchBytes = (kScratchRecords + 1) * kPartials * 8 + 256;
static __device__ __align__(256) char scratch[kScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// The device address of `scratch` on the current device. In host code the
// array's name is only a stand-in for the symbol, not a device address: it is
// resolved once per device with hipGetSymbolAddress, with that device current,
// and only the resolved pointer is handed to kernels.
int scratch_address(void** out) {
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(LB_EHIP, "device index beyond the scratch table");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return fail(LB_EHIP, "hipGetSymbolAddress returned no address for the scratch");
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return LB_OK;
}
}  // namespace

struct Member {
    lb_params p;
    Layout L;
    char* base = nullptr;  // arena
    View view{};
    View* d_view = nullptr;
    std::vector<uint8_t> solid;  // host copy (nx*ny)
    std::vector<double> dphi;    // host copy (nx*ny)
    int64_t n_fluid = 0;
};

struct Group {
    std::vector<Member> m;
    hipStream_t stream = nullptr;
    hipStream_t capture_stream = nullptr;
    char* alloc = nullptr;  // owned device memory (null for caller buffers)
    int parity = 0;
    int64_t step = 0;
    int block_x = 256;
    int rows = 32;
    // batched launch data (members > 1)
    Tile* d_tiles = nullptr;
    int32_t* d_first = nullptr;  // n+1 tile offsets per member
    double* d_partials = nullptr;
    double* d_diag = nullptr;
    int32_t* d_flag = nullptr;
    View* d_views = nullptr;
    int n_tiles = 0;             // logical tiles the allocation holds (largest tiling)
    int n_step_slots = 0;        // workgroups of a stepwise batch launch (table entries)
    int step_slots_max = 0;      // entries the stepwise table holds
    char* batch_alloc = nullptr;
    // Captured graphs, one per (window length 2^l, parity of its first step,
    // whether its first step carries the periodic check): index (l*2 + parity)*2 + check.
    hipGraphExec_t graph[kGraphLens * 4] = {};
    bool batched = false;
    bool any_walls = false;  // a batch member uses lattice-node bounce-back
    // persistent schedule of a batch (sweep_persistent_kernel)
    int schedule = LB_SCHEDULE_STEPWISE;
    uint32_t spin_limit = kDefaultSpinLimit;
    Tile* d_ptiles = nullptr;    // tiles in logical order (member-major, row-major)
    int32_t* d_deps = nullptr;   // kPersistDeps logical tile ids per tile (-1 = none)
    int32_t* d_sync = nullptr;   // [0] error flag, [1] claim counter, [2..] done per tile
    int persist_grid = 0;        // workgroups of a persistent launch
    int max_deps = 0;            // most tiles one tile depends on, current tiling
};

struct lb_handle {
    Group g;
};
struct lb_batch {
    Group g;
};

namespace {

bool is_finite(double v) { return std::isfinite(v); }

int validate_params(const lb_params* p) {
    if (!p) return fail(LB_EINVAL, "params is NULL");
    if (p->nx < 3 || p->ny < 3) return fail(LB_EINVAL, "nx and ny must be >= 3");
    if (p->nx > (1 << 24) || p->ny > (1 << 24) || (int64_t)p->nx * p->ny > (int64_t)1 << 34)
        return fail(LB_EINVAL, "lattice too large");
    const double vals[] = {p->A, p->B, p->kappa, p->Gamma, p->tau_alpha,
                           p->tau_beta, p->tau_phi, p->rho_ref};
    for (double v : vals)
        if (!is_finite(v)) return fail(LB_EINVAL, "non-finite parameter");
    if (!(p->tau_alpha > 0.5) || !(p->tau_beta > 0.5) || !(p->tau_phi > 0.5))
        return fail(LB_EINVAL, "tau_alpha, tau_beta and tau_phi must exceed 1/2");
    if (!(p->rho_ref > 0)) return fail(LB_EINVAL, "rho_ref must be positive");
    if (p->collision != LB_BGK && p->collision != LB_MRT)
        return fail(LB_EINVAL, "collision must be LB_BGK or LB_MRT");
    if (p->storage < LB_F64 || p->storage > LB_F32C)
        return fail(LB_EINVAL, "unknown storage format");
    if ((p->storage == LB_F64C || p->storage == LB_F32C) && p->tau_phi != 1.0)
        return fail(LB_EINVAL, "the compressed-g formats need tau_phi = 1");
    if ((p->zero_u_feq != 0 && p->zero_u_feq != 1) || (p->zero_u_geq != 0 && p->zero_u_geq != 1))
        return fail(LB_EINVAL, "zero_u flags must be 0 or 1");
    if (p->diag_every < 0) return fail(LB_EINVAL, "diag_every must be >= 0");
    if (p->tau_clamp != 0 && p->tau_clamp != 1) return fail(LB_EINVAL, "tau_clamp must be 0 or 1");
    if (p->inplace != 0 && p->inplace != 1) return fail(LB_EINVAL, "inplace must be 0 or 1");
    if (p->inplace && p->storage != LB_F64 && p->storage != LB_F32)
        return fail(LB_EINVAL, "in-place update is available for LB_F64 and LB_F32");
    if (p->tau_lut < 0 || p->tau_lut == 1 || p->tau_lut > (1 << 24))
        return fail(LB_EINVAL, "tau_lut must be 0 or 2 .. 2^24");
    if (p->bounce != LB_MIDLINK && p->bounce != LB_LATTICE_NODE)
        return fail(LB_EINVAL, "bounce must be LB_MIDLINK or LB_LATTICE_NODE");
    if (p->bounce == LB_LATTICE_NODE &&
        (p->inplace || (p->storage != LB_F64 && p->storage != LB_F32)))
        return fail(LB_EINVAL, "lattice-node bounce-back is available for LB_F64 and LB_F32 "
                               "with inplace = 0");
    // One row block of the populations is addressed through a buffer
    // descriptor with a 32-bit record count.
    if ((int64_t)((p->nx + 63) / 64) * 64 * 18 * 8 >= ((int64_t)1 << 31))
        return fail(LB_EINVAL, "nx too large");
    return LB_OK;
}

int validate_inputs(const lb_params* p, const uint8_t* solid, const double* dphi,
                    const double* phi0, const double* rho0, const double* ux0, const double* uy0,
                    int64_t* n_fluid) {
    if (!solid || !phi0) return fail(LB_EINVAL, "solid and phi0 are required");
    const int nx = p->nx, ny = p->ny;
    int64_t nf = 0;
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            const int64_t h = (int64_t)y * nx + x;
            if (solid[h]) {
                if (dphi && !is_finite(dphi[h])) return fail(LB_EINVAL, "non-finite wall_dphi");
                continue;
            }
            ++nf;
            if (!is_finite(phi0[h])) return fail(LB_EINVAL, "non-finite phi0");
            if (rho0 && !(is_finite(rho0[h]) && rho0[h] > 0))
                return fail(LB_EINVAL, "rho0 must be finite and positive at fluid nodes");
            if ((ux0 && !is_finite(ux0[h])) || (uy0 && !is_finite(uy0[h])))
                return fail(LB_EINVAL, "non-finite initial velocity");
            bool enclosed = true;
            for (int i = 1; i < 9; ++i) {
                const int xs = (x + kEX[i] + nx) % nx, ys = (y + kEY[i] + ny) % ny;
                if (!solid[(int64_t)ys * nx + xs]) enclosed = false;
            }
            if (enclosed) return fail(LB_EINVAL, "a fluid node has no fluid neighbour");
        }
    *n_fluid = nf;
    return LB_OK;
}

std::vector<uint8_t> make_nbr(const lb_params* p, const Layout& L, const uint8_t* solid) {
    const int nx = p->nx, ny = p->ny;
    std::vector<uint8_t> nbr((size_t)L.plane, 0xFF);
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            const int64_t h = (int64_t)y * nx + x;
            uint8_t b = 0xFF;
            if (!solid[h]) {
                b = 0;
                for (int i = 1; i < 9; ++i) {
                    const int xs = (x - kEX[i] + nx) % nx, ys = (y - kEY[i] + ny) % ny;
                    if (solid[(int64_t)ys * nx + xs]) b |= (uint8_t)(1u << (i - 1));
                }
            }
            nbr[(size_t)y * L.pitch + x] = b;
        }
    return nbr;
}

std::vector<uint8_t> make_grec(const lb_params* p, const Layout& L, const uint8_t* solid) {
    const int nx = p->nx, ny = p->ny;
    std::vector<uint8_t> grec((size_t)L.plane, 0);
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            if (!solid[(int64_t)y * nx + x]) continue;
            uint8_t b = 0;
            for (int m = 1; m < 9; ++m) {
                const int xs = (x + kEX[m] + nx) % nx, ys = (y + kEY[m] + ny) % ny;
                if (!solid[(int64_t)ys * nx + xs]) b |= (uint8_t)(1u << (m - 1));
            }
            grec[(size_t)y * L.pitch + x] = b;
        }
    return grec;
}

int upload_dphi(Member& mb, const double* dphi, hipStream_t st) {
    const lb_params& p = mb.p;
    const Layout& L = mb.L;
    mb.dphi.assign((size_t)p.nx * p.ny, 0.0);
    for (int64_t h = 0; h < (int64_t)p.nx * p.ny; ++h)
        if (mb.solid[h] && dphi) mb.dphi[h] = dphi[h];
    char* dst = mb.base + L.off_dphi;
    if (p.storage == LB_F64 || p.storage == LB_F64C) {
        std::vector<double> d((size_t)L.plane, 0.0);
        for (int y = 0; y < p.ny; ++y)
            for (int x = 0; x < p.nx; ++x) d[(size_t)y * L.pitch + x] = mb.dphi[(size_t)y * p.nx + x];
        HIPCHK(hipMemcpyAsync(dst, d.data(), d.size() * 8, hipMemcpyHostToDevice, st));
        HIPCHK(hipStreamSynchronize(st));
    } else {
        std::vector<float> d((size_t)L.plane, 0.0f);
        for (int y = 0; y < p.ny; ++y)
            for (int x = 0; x < p.nx; ++x)
                d[(size_t)y * L.pitch + x] = (float)mb.dphi[(size_t)y * p.nx + x];
        HIPCHK(hipMemcpyAsync(dst, d.data(), d.size() * 4, hipMemcpyHostToDevice, st));
        HIPCHK(hipStreamSynchronize(st));
    }
    return LB_OK;
}

// Initialise one member whose arena base is already set.
int init_member(Member& mb, const lb_params* p, const uint8_t* solid, const double* dphi,
                const double* phi0, const double* rho0, const double* ux0, const double* uy0,
                hipStream_t st) {
    mb.p = *p;
    const Layout& L = mb.L;
    const int nx = p->nx, ny = p->ny;
    const size_t n = (size_t)nx * ny;
    HIPCHK(launch_fill(mb.base, 0, L.total, st));
    mb.solid.assign(solid, solid + n);
    for (auto& s : mb.solid) s = s ? 1 : 0;
    const std::vector<uint8_t> nbr = make_nbr(p, L, mb.solid.data());
    const std::vector<uint8_t> grec = make_grec(p, L, mb.solid.data());
    HIPCHK(hipMemcpyAsync(mb.base + L.off_nbr, nbr.data(), nbr.size(), hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(mb.base + L.off_grec, grec.data(), grec.size(), hipMemcpyHostToDevice, st));
    HIPCHK(hipStreamSynchronize(st));
    int rc = upload_dphi(mb, dphi, st);
    if (rc) return rc;

    View& v = mb.view;
    v = View{};
    v.nx = nx;
    v.ny = ny;
    v.pitch = L.pitch;
    v.plane = L.plane;
    v.row_bytes = (int64_t)L.row_bytes;
    v.g0_offset = (int64_t)L.g0_offset;
    v.buf[0] = mb.base + L.off_buf0;
    v.buf[1] = mb.base + L.off_buf1;
    v.band = p->inplace ? mb.base + L.off_band : nullptr;
    v.inplace = p->inplace;
    v.tau_lut = p->tau_lut;
    v.bounce = p->bounce;
    v.tau_step = p->tau_lut > 1 ? (p->tau_alpha - p->tau_beta) / (p->tau_lut - 1) : 0.0;
    v.nbr = reinterpret_cast<const uint8_t*>(mb.base + L.off_nbr);
    v.grec = reinterpret_cast<const uint8_t*>(mb.base + L.off_grec);
    v.dphi = mb.base + L.off_dphi;
    v.A = p->A;
    v.B = p->B;
    v.kappa = p->kappa;
    v.Gamma = p->Gamma;
    v.tau_alpha = p->tau_alpha;
    v.tau_beta = p->tau_beta;
    v.inv_tau_phi = 1.0 / p->tau_phi;
    // Rest state of the model at rho_ref in either bulk phase phi = +-1 (p0 is
    // even in phi): r_i = w_i p0 for i >= 1, r_0 = rho_ref - (5/3) p0. The
    // formats other than FP64 store f_i - r_i.
    v.rho_ref = p->rho_ref;
    v.p0_ref = p->rho_ref / 3.0 + 0.5 * p->A + 0.75 * p->B;
    v.zero_u_feq = p->zero_u_feq;
    v.zero_u_geq = p->zero_u_geq;
    v.storage = p->storage;
    v.collision = p->collision;
    v.tau_clamp = p->tau_clamp;
    mb.d_view = reinterpret_cast<View*>(mb.base + L.off_view);
    HIPCHK(hipMemcpyAsync(mb.d_view, &v, sizeof(View), hipMemcpyHostToDevice, st));

    // Stage the initial fields (compact FP64, defaults filled) in buf[1].
    std::vector<double> stage(4 * n);
    for (size_t h = 0; h < n; ++h) {
        stage[h] = mb.solid[h] ? 0.0 : phi0[h];
        stage[n + h] = rho0 ? rho0[h] : p->rho_ref;
        stage[2 * n + h] = ux0 ? ux0[h] : 0.0;
        stage[3 * n + h] = uy0 ? uy0[h] : 0.0;
    }
    if (p->inplace) {
        // rho0, ux0, uy0 go to each node's own slots of planes 1..3 (FP64) or,
        // as low and high words, 1..6 (FP32); phi0 then stays in the band
        // plane. Each field crosses to the device as one contiguous copy into
        // the band plane and is spread over the slots by a device-to-device 2D
        // copy: a 2D copy from pageable host memory would move the short rows
        // one by one.
        char* band = reinterpret_cast<char*>(v.band);
        std::vector<uint32_t> words;
        for (int q = 0; q < 3; ++q) {
            const double* src = stage.data() + (size_t)(q + 1) * n;
            if (p->storage == LB_F64) {
                HIPCHK(hipMemcpyAsync(band, src, n * 8, hipMemcpyHostToDevice, st));
                HIPCHK(hipMemcpy2DAsync(v.buf[0] + (size_t)(1 + q) * L.pitch * 8, L.row_bytes, band,
                                        (size_t)nx * 8, (size_t)nx * 8, (size_t)ny,
                                        hipMemcpyDeviceToDevice, st));
            } else {
                words.resize(2 * n);
                for (size_t h = 0; h < n; ++h) {
                    uint64_t u;
                    std::memcpy(&u, src + h, 8);
                    words[h] = (uint32_t)u;
                    words[n + h] = (uint32_t)(u >> 32);
                }
                HIPCHK(hipMemcpyAsync(band, words.data(), 2 * n * 4, hipMemcpyHostToDevice, st));
                for (int half = 0; half < 2; ++half)
                    HIPCHK(hipMemcpy2DAsync(v.buf[0] + (size_t)(1 + 2 * q + half) * L.pitch * 4,
                                            L.row_bytes, band + (size_t)half * n * 4, (size_t)nx * 4,
                                            (size_t)nx * 4, (size_t)ny, hipMemcpyDeviceToDevice, st));
            }
            HIPCHK(hipStreamSynchronize(st));  // the band plane and words are reused
        }
        HIPCHK(hipMemcpyAsync(band, stage.data(), n * 8, hipMemcpyHostToDevice, st));
        const double* d_phi0 = reinterpret_cast<const double*>(v.band);
        HIPCHK(launch_init_state(v, d_phi0, nullptr, nullptr, nullptr, st));
        HIPCHK(hipStreamSynchronize(st));
        return LB_OK;
    }
    double* d_stage = reinterpret_cast<double*>(v.buf[1]);
    HIPCHK(hipMemcpyAsync(d_stage, stage.data(), stage.size() * 8, hipMemcpyHostToDevice, st));
    HIPCHK(launch_init_state(v, d_stage, d_stage + n, d_stage + 2 * n, d_stage + 3 * n, st));
    HIPCHK(hipStreamSynchronize(st));
    return LB_OK;
}

void destroy_graphs(Group& g) {
    for (auto& e : g.graph)
        if (e) {
            (void)hipGraphExecDestroy(e);
            e = nullptr;
        }
}

int check_tuning(int bx, int rows) {
    if (bx != 64 && bx != 128 && bx != 256 && bx != 512 && bx != 1024)
        return fail(LB_EINVAL, "block_x must be 64, 128, 256, 512 or 1024");
    if (rows < 1 || rows > 1024) return fail(LB_EINVAL, "rows_per_block must be in 1..1024");
    return LB_OK;
}

// Strip height of batch member `mb` under tuning (bx, rows): a member narrower
// than bx gets strips taller in proportion, so its tiles hold about as many
// nodes as the others' (bx x rows); never more than the member's height.
int member_rows(const lb_params& p, int bx, int rows) {
    const int64_t widen = p.nx < bx ? (bx + p.nx - 1) / p.nx : 1;
    return (int)std::min<int64_t>((int64_t)rows * widen, p.ny);
}

// Tile tables of a batched group for the current tuning: the stepwise table in
// XCD-aware order, the logical table (member-major, row-major) of the
// persistent schedule, and each tile's dependencies: the tiles of the same
// member holding a column and a row that its step reads (itself included).
int build_tiles(Group& g) {
    g.max_deps = 0;
    std::vector<Tile> logical;
    std::vector<int32_t> first, deps;
    for (size_t k = 0; k < g.m.size(); ++k) {
        const lb_params& p = g.m[k].p;
        const int rows = member_rows(p, g.block_x, g.rows);
        first.push_back((int32_t)logical.size());
        const int tx = (p.nx + g.block_x - 1) / g.block_x;
        const int ty = (p.ny + rows - 1) / rows;
        const int base = (int)logical.size();
        for (int j = 0; j < ty; ++j)
            for (int i = 0; i < tx; ++i) {
                const int y0 = j * rows, y1 = std::min((j + 1) * rows, p.ny);
                logical.push_back(Tile{(int32_t)k, i, j, (int32_t)logical.size(), y0, y1});
                // Column and strip indices reached by the tile's step: its pulls
                // and phi stencil with ghosts reach three nodes beyond its
                // columns (wrapped lanes included) and rows, periodically.
                const int x0 = i * g.block_x, x1 = std::min(x0 + g.block_x, p.nx);
                std::vector<int> cols, strips;
                for (int c = x0 - 3; c <= x1 + 2; ++c) {
                    const int ci = ((c % p.nx) + p.nx) % p.nx / g.block_x;
                    if (std::find(cols.begin(), cols.end(), ci) == cols.end()) cols.push_back(ci);
                }
                for (int r = y0 - 3; r <= y1 + 2; ++r) {
                    const int sj = std::min(((r % p.ny) + p.ny) % p.ny / rows, ty - 1);
                    if (std::find(strips.begin(), strips.end(), sj) == strips.end())
                        strips.push_back(sj);
                }
                int nd = 0;
                for (int sj : strips)
                    for (int ci : cols) {
                        if (nd < kPersistDeps) deps.push_back(base + sj * tx + ci);
                        ++nd;
                    }
                for (int q = nd; q < kPersistDeps; ++q) deps.push_back(-1);
                g.max_deps = std::max(g.max_deps, nd);
            }
    }
    first.push_back((int32_t)logical.size());
    // Stepwise table: workgroup b runs on XCD b % 8. Members are dealt to the
    // 8 XCDs, largest first, each to the XCD with the least work so far (a
    // tile's work: its rows times the tile width, idle lanes included), so a
    // member's neighbouring tiles share one L2 and the XCDs get equal work; a
    // member with more work than an eighth of the total is first cut into
    // contiguous runs of its tiles (row-major) of equal work, at most an eighth
    // each, and the runs are dealt the same way. Each XCD then takes its tiles
    // largest first. XCD k's i-th tile is entry 8 i + k; shorter lists are
    // padded with empty entries (member -1).
    const int n = (int)logical.size();
    std::vector<int> morder(g.m.size());
    std::vector<int64_t> mwork(g.m.size(), 0);
    for (size_t k = 0; k < g.m.size(); ++k) morder[k] = (int)k;
    for (const Tile& t : logical) mwork[t.member] += (int64_t)(t.y1 - t.y0) * g.block_x;
    std::stable_sort(morder.begin(), morder.end(),
                     [&](int a, int b) { return mwork[a] > mwork[b]; });
    int64_t work = 0;
    for (int64_t w : mwork) work += w;
    const int64_t share = (work + 7) / 8;
    std::vector<std::vector<Tile>> bins(8);
    int64_t load[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int k : morder) {
        const int64_t runs = share > 0 ? std::max<int64_t>(1, (mwork[k] + share - 1) / share) : 1;
        int64_t acc = 0;
        int run = -1, x = 0;
        for (int i = first[k]; i < first[k + 1]; ++i) {
            const int64_t w = (int64_t)(logical[i].y1 - logical[i].y0) * g.block_x;
            // the run holding the middle of this tile's work
            const int r = (int)std::min<int64_t>(runs - 1, (2 * acc + w) * runs / (2 * mwork[k]));
            if (r != run) {
                run = r;
                x = (int)(std::min_element(load, load + 8) - load);
            }
            bins[x].push_back(logical[i]);
            load[x] += w;
            acc += w;
        }
    }
    size_t max_len = 0;
    for (auto& bin : bins) {
        std::stable_sort(bin.begin(), bin.end(), [](const Tile& a, const Tile& b) {
            return a.y1 - a.y0 > b.y1 - b.y0;
        });
        max_len = std::max(max_len, bin.size());
    }
    std::vector<Tile> tiles(8 * max_len, Tile{-1, 0, 0, -1, 0, 0});
    for (int x = 0; x < 8; ++x)
        for (size_t i = 0; i < bins[x].size(); ++i) tiles[8 * i + x] = bins[x][i];
    if ((size_t)n > (size_t)g.n_tiles || tiles.size() > (size_t)g.step_slots_max)
        return fail(LB_EINVAL, "tile table too small for this tuning");
    g.n_step_slots = (int)tiles.size();
    HIPCHK(hipMemcpyAsync(g.d_tiles, tiles.data(), tiles.size() * sizeof(Tile),
                          hipMemcpyHostToDevice, g.stream));
    HIPCHK(hipMemcpyAsync(g.d_ptiles, logical.data(), logical.size() * sizeof(Tile),
                          hipMemcpyHostToDevice, g.stream));
    HIPCHK(hipMemcpyAsync(g.d_deps, deps.data(), deps.size() * 4, hipMemcpyHostToDevice,
                          g.stream));
    HIPCHK(hipMemcpyAsync(g.d_first, first.data(), first.size() * 4, hipMemcpyHostToDevice,
                          g.stream));
    HIPCHK(hipStreamSynchronize(g.stream));
    return LB_OK;
}

// Whether the batch can run the persistent schedule with its tuning: a tile's
// reach (three nodes) must stay within its neighbouring tiles.
bool persistent_ok(const Group& g, std::string* why) {
    if (g.any_walls) {
        if (why) *why = "lattice-node bounce-back members need the stepwise schedule";
        return false;
    }
    if (g.block_x != 128 && g.block_x != 256 && g.block_x != 512) {
        if (why) *why = "the persistent schedule takes block_x 128, 256 or 512";
        return false;
    }
    for (const auto& mb : g.m) {
        const int rows = member_rows(mb.p, g.block_x, g.rows);
        if (rows < 3 && rows < mb.p.ny) {
            if (why) *why = "the persistent schedule needs strips of at least 3 rows";
            return false;
        }
    }
    if (g.max_deps > kPersistDeps) {
        if (why) *why = "a tile of this tiling depends on more tiles than the persistent "
                        "schedule tracks";
        return false;
    }
    return true;
}

// Workgroups of a persistent launch: as many as fit on the device at once.
int persistent_grid(Group& g) {
    int dev = 0, cus = 0, per_cu = 0;
    HIPCHK(hipGetDevice(&dev));
    HIPCHK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    const lb_params& p = g.m[0].p;
    HIPCHK(persistent_occupancy(p.storage, p.collision, g.block_x, p.tau_phi == 1.0, &per_cu));
    g.persist_grid = std::max(1, cus * std::max(1, per_cu));
    return LB_OK;
}

int current_tiles(const Group& g) {
    int n = 0;
    for (const auto& mb : g.m) {
        const int rows = g.batched ? member_rows(mb.p, g.block_x, g.rows) : g.rows;
        n += ((mb.p.nx + g.block_x - 1) / g.block_x) * ((mb.p.ny + rows - 1) / rows);
    }
    return n;
}

// Enqueue `len` timesteps of a batch on the persistent schedule, starting at
// `parity`: clear the claim counter and the per-tile step counts, then one
// persistent launch.
hipError_t enqueue_persistent(Group& g, int len, int parity, hipStream_t st) {
    const Member& m0 = g.m[0];
    const int nt = current_tiles(g);
    hipError_t e = launch_fill(g.d_sync + 1, 0, (size_t)(nt + 1) * 4, st);
    if (e != hipSuccess) return e;
    // No more workgroups than two steps' tiles: further ones could only wait.
    const int grid = (int)std::min<int64_t>(g.persist_grid, (int64_t)nt * std::min(len, 2));
    return launch_persistent(m0.p.storage, m0.p.collision, g.block_x, m0.p.tau_phi == 1.0,
                             g.d_views, g.d_ptiles, g.d_deps, nt, len, parity, grid, g.d_sync + 2,
                             reinterpret_cast<uint32_t*>(g.d_sync + 1), g.d_sync, g.spin_limit,
                             st);
}

// Enqueue one timestep of every member on stream st.
hipError_t enqueue_one(Group& g, bool diag, int parity, hipStream_t st) {
    const Member& m0 = g.m[0];
    if (!g.batched) {
        const Layout& L = m0.L;
        const int gx = (m0.p.nx + g.block_x - 1) / g.block_x;
        const int gy = (m0.p.ny + g.rows - 1) / g.rows;
        double* partials = reinterpret_cast<double*>(m0.base + L.off_partials);
        if (m0.p.inplace) {
            hipError_t e = launch_band(m0.p.storage, m0.p.tau_phi == 1.0, m0.d_view, m0.p.nx,
                                       m0.p.ny, g.block_x, g.rows, parity, st);
            if (e != hipSuccess) return e;
        }
        hipError_t e = launch_sweep(m0.p.storage, m0.p.collision, g.block_x, diag,
                                    m0.p.tau_phi == 1.0, m0.p.inplace != 0, m0.d_view, nullptr, 0,
                                    gx, gy, g.rows, parity, partials, st);
        if (e == hipSuccess && m0.p.bounce == LB_LATTICE_NODE)
            e = launch_walls(m0.p.storage, g.block_x, m0.d_view, nullptr, 0, gx, gy, g.rows,
                             parity, st);
        if (e != hipSuccess || !diag) return e;
        return launch_finalize(nullptr, nullptr, 1, gx * gy, partials,
                               reinterpret_cast<double*>(m0.base + L.off_diag),
                               reinterpret_cast<int32_t*>(m0.base + L.off_flag), st);
    }
    const int nt = g.n_step_slots;
    hipError_t e = launch_sweep(m0.p.storage, m0.p.collision, g.block_x, diag,
                                m0.p.tau_phi == 1.0, false, g.d_views, g.d_tiles, nt, 0, 0, g.rows,
                                parity, g.d_partials, st);
    if (e == hipSuccess && g.any_walls)
        e = launch_walls(m0.p.storage, g.block_x, g.d_views, g.d_tiles, nt, 0, 0, g.rows, parity,
                         st);
    if (e != hipSuccess || !diag) return e;
    return launch_finalize(g.d_tiles, g.d_first, (int)g.m.size(), 0, g.d_partials, g.d_diag,
                           g.d_flag, st);
}

// Enqueue `len` timesteps starting at `parity`, the first with the periodic
// check when `check`: one launch per step, or, for a batch on the persistent
// schedule, the checked step (if any) and then one persistent launch.
hipError_t enqueue_window(Group& g, int len, int parity, bool check, hipStream_t st) {
    if (g.batched && g.schedule == LB_SCHEDULE_PERSISTENT) {
        int done = 0;
        if (check) {
            hipError_t e = enqueue_one(g, true, parity, st);
            if (e != hipSuccess) return e;
            done = 1;
        }
        if (done < len) return enqueue_persistent(g, len - done, (parity + done) & 1, st);
        return hipSuccess;
    }
    hipError_t ce = hipSuccess;
    for (int s = 0; s < len && ce == hipSuccess; ++s)
        ce = enqueue_one(g, check && s == 0, (parity + s) & 1, st);
    return ce;
}

// Capture `len` timesteps starting at `parity`, the first with the periodic
// check when `check`, into one executable graph.
int capture_graph(Group& g, int len, int parity, bool check, hipGraphExec_t* out) {
    Range r("lb graph capture");
    if (!g.capture_stream)
        HIPCHK(hipStreamCreateWithFlags(&g.capture_stream, hipStreamNonBlocking));
    HIPCHK(hipStreamBeginCapture(g.capture_stream, hipStreamCaptureModeRelaxed));
    hipError_t ce = enqueue_window(g, len, parity, check, g.capture_stream);
    hipGraph_t graph = nullptr;
    hipError_t ee = hipStreamEndCapture(g.capture_stream, &graph);
    if (ce != hipSuccess || ee != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        return fail(LB_EHIP, std::string("graph capture failed: ") +
                                 hipGetErrorString(ce != hipSuccess ? ce : ee));
    }
    hipError_t ie = hipGraphInstantiate(out, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ie != hipSuccess) {
        *out = nullptr;
        return fail(LB_EHIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(ie));
    }
    // Move the graph's launch data to the device now, not at its first replay.
    HIPCHK(hipGraphUpload(*out, g.stream));
    return LB_OK;
}

// Every step runs from a captured graph. A call is cut into windows of 2^l
// steps (at most kGraphSteps) whose only periodic check, if any, is at their
// first step; each window replays the graph of its length, starting parity and
// check. All graphs of a group are captured together the first time it steps
// (and again after a change of tiles), so that a later call of any length and
// phase replays graphs only.
int group_step(Group& g, int64_t nsteps) {
    if (nsteps < 0) return fail(LB_EINVAL, "nsteps must be >= 0");
    if (nsteps == 0) return LB_OK;
    const int de = g.m[0].p.diag_every;
    if (!g.graph[0]) {
        for (int l = 0; l < kGraphLens; ++l)
            for (int par = 0; par < 2; ++par)
                for (int chk = 0; chk < (de > 0 ? 2 : 1); ++chk) {
                    int rc = capture_graph(g, 1 << l, par, chk != 0,
                                           &g.graph[(l * 2 + par) * 2 + chk]);
                    if (rc) {
                        destroy_graphs(g);
                        return rc;
                    }
                }
    }
    int64_t left = nsteps;
    while (left > 0) {
        int64_t lim = std::min<int64_t>(left, kGraphSteps);
        if (de > 0) lim = std::min<int64_t>(lim, de - g.step % de);
        int l = 0;
        while ((int64_t)2 << l <= lim) ++l;
        const bool chk = de > 0 && g.step % de == 0;
        {
            Range r("lb graph replay");
            HIPCHK(hipGraphLaunch(g.graph[(l * 2 + g.parity) * 2 + (chk ? 1 : 0)], g.stream));
        }
        const int len = 1 << l;
        g.parity = (g.parity + len) & 1;
        g.step += len;
        left -= len;
    }
    return LB_OK;
}

// Whether every persistent window of a batch enqueued so far ran to completion
// (it waits for them): a window whose wait gave up leaves the state invalid,
// which every read of a batch reports.
int check_windows(Group& g) {
    if (g.batched && g.d_sync) {
        int32_t err = 0;
        HIPCHK(hipMemcpyAsync(&err, g.d_sync, 4, hipMemcpyDeviceToHost, g.stream));
        HIPCHK(hipStreamSynchronize(g.stream));
        if (err)
            return fail(LB_EHIP, "persistent schedule: a wait for a neighbouring tile exceeded "
                                 "its poll limit; the state is not valid");
    }
    return LB_OK;
}

int check_flag(Group& g) {
    if (int rc = check_windows(g)) return rc;
    for (size_t k = 0; k < g.m.size(); ++k) {
        int32_t flag = 0;
        const int32_t* src = g.batched ? g.d_flag + k
                                       : reinterpret_cast<const int32_t*>(g.m[k].base + g.m[k].L.off_flag);
        HIPCHK(hipMemcpyAsync(&flag, src, 4, hipMemcpyDeviceToHost, g.stream));
        HIPCHK(hipStreamSynchronize(g.stream));
        if (flag) return fail(LB_ENUMERIC, "a periodic diagnostic found a non-finite value");
    }
    return LB_OK;
}

// Device scratch between steps: the other population buffer, or in place the
// band plane (at least 8 bytes per node).
std::pair<char*, size_t> scratch_of(const Group& g, const Member& mb) {
    if (mb.p.inplace) return {mb.base + mb.L.off_band, round_up((size_t)mb.L.plane * 8, 256)};
    return {mb.view.buf[g.parity ^ 1], mb.L.buf_bytes};
}

int read_fields(Group& g, int k, double* phi, double* rho, double* ux, double* uy) {
    Member& mb = g.m[k];
    const int64_t n = (int64_t)mb.p.nx * mb.p.ny;
    const auto sc = scratch_of(g, mb);
    double* stage = reinterpret_cast<double*>(sc.first);
    const int64_t chunk = std::min<int64_t>(n, (int64_t)(sc.second / 32));
    double* outs[4] = {phi, rho, ux, uy};
    for (int64_t first = 0; first < n; first += chunk) {
        const int64_t cnt = std::min(chunk, n - first);
        HIPCHK(launch_moments(mb.view, g.parity, first, cnt, stage, nullptr, 0, 0, 0, g.stream));
        for (int q = 0; q < 4; ++q)
            if (outs[q])
                HIPCHK(hipMemcpyAsync(outs[q] + first, stage + q * cnt, cnt * 8,
                                      hipMemcpyDeviceToHost, g.stream));
        HIPCHK(hipStreamSynchronize(g.stream));
    }
    return LB_OK;
}

int read_populations(Group& g, int k, double* f, double* gg) {
    Member& mb = g.m[k];
    const size_t n = (size_t)mb.p.nx * mb.p.ny;
    double* stage = reinterpret_cast<double*>(scratch_of(g, mb).first);
    for (int pl = 0; pl < 18; ++pl) {
        double* out = pl < 9 ? f : gg;
        if (!out) continue;
        HIPCHK(launch_read_plane(mb.view, g.parity, pl, stage, g.stream));
        HIPCHK(hipMemcpyAsync(out + (size_t)(pl % 9) * n, stage, n * 8, hipMemcpyDeviceToHost,
                              g.stream));
        HIPCHK(hipStreamSynchronize(g.stream));
    }
    return LB_OK;
}

// Sums over fluid nodes: out[0..5] = sum rho, sum phi, kinetic, max |u|, count,
// sum (1+phi)/2 for x_lo <= x < x_hi.
int reduce_member(Group& g, int k, int32_t x_lo, int32_t x_hi, double out[6]) {
    Member& mb = g.m[k];
    const Layout& L = mb.L;
    double* partials = reinterpret_cast<double*>(mb.base + L.off_partials);
    double* diag = reinterpret_cast<double*>(mb.base + L.off_diag);
    int32_t* flag = reinterpret_cast<int32_t*>(mb.base + L.off_flag);
    const int nrec = (int)(((int64_t)mb.p.nx * mb.p.ny + 255) / 256);
    HIPCHK(launch_moments(mb.view, g.parity, 0, (int64_t)mb.p.nx * mb.p.ny, nullptr, partials,
                          (int)L.n_partials, x_lo, x_hi, g.stream));
    // A separate scratch flag keeps the sticky periodic flag untouched.
    HIPCHK(launch_finalize(nullptr, nullptr, 1, nrec, partials, diag, flag + 1, g.stream));
    double rec[kPartials];
    HIPCHK(hipMemcpyAsync(rec, diag, sizeof(rec), hipMemcpyDeviceToHost, g.stream));
    HIPCHK(hipStreamSynchronize(g.stream));
    for (int q = 0; q < 6; ++q) out[q] = rec[q];
    return LB_OK;
}

// Kasa circle fit of the crossings, in FP64 on the host after sorting by link,
// so the result does not depend on the order in which the GPU found them.
int contact_angle(Group& g, int k, double x_lo, double x_hi, double y_lo, double y_hi,
                  double y_wall, int wall_dir, double* theta, double* xc_out, double* yc_out,
                  double* r_out, int64_t* np_out) {
    if (!theta) return fail(LB_EINVAL, "theta_deg is NULL");
    if (wall_dir != 1 && wall_dir != -1) return fail(LB_EINVAL, "wall_dir must be +1 or -1");
    if (!(x_hi > x_lo) || !(y_hi >= y_lo)) return fail(LB_EINVAL, "empty window");
    Member& mb = g.m[k];
    const int nx = mb.p.nx, ny = mb.p.ny;
    const Layout& L = mb.L;
    unsigned long long* counter = reinterpret_cast<unsigned long long*>(mb.base + L.off_counter);
    const auto sc = scratch_of(g, mb);
    void* pts = sc.first;
    const int64_t cap = (int64_t)(sc.second / sizeof(Crossing));
    HIPCHK(launch_fill(counter, 0, 8, g.stream));
    HIPCHK(launch_crossings(mb.view, g.parity, pts, cap, counter, g.stream));
    unsigned long long count = 0;
    HIPCHK(hipMemcpyAsync(&count, counter, 8, hipMemcpyDeviceToHost, g.stream));
    HIPCHK(hipStreamSynchronize(g.stream));
    if ((int64_t)count > cap) return fail(LB_ENOMEM, "too many interface crossings");
    std::vector<Crossing> c(count);
    if (count) {
        HIPCHK(hipMemcpyAsync(c.data(), pts, count * sizeof(Crossing), hipMemcpyDeviceToHost,
                              g.stream));
        HIPCHK(hipStreamSynchronize(g.stream));
    }
    std::sort(c.begin(), c.end(), [](const Crossing& a, const Crossing& b) { return a.key < b.key; });
    const double cx = 0.5 * (x_lo + x_hi), cy = 0.5 * (y_lo + y_hi);
    std::vector<double> px, py, ex, ey;
    for (const Crossing& q : c) {
        const uint64_t node = q.key >> 2;
        const int axis = (int)((q.key >> 1) & 1);
        const bool base_pos = q.key & 1;
        const double bx = (double)(node % (uint64_t)nx), by = (double)(node / (uint64_t)nx);
        double x = bx + (axis == 0 ? q.t : 0.0), y = by + (axis == 1 ? q.t : 0.0);
        double qx = base_pos ? bx : bx + (axis == 0), qy = base_pos ? by : by + (axis == 1);
        const double sx = nx * std::nearbyint((x - cx) / nx);
        const double sy = ny * std::nearbyint((y - cy) / ny);
        x -= sx; qx -= sx;
        y -= sy; qy -= sy;
        if (x >= x_lo && x < x_hi && y >= y_lo && y <= y_hi) {
            px.push_back(x); py.push_back(y); ex.push_back(qx); ey.push_back(qy);
        }
    }
    const size_t m = px.size();
    if (np_out) *np_out = (int64_t)m;
    if (m < 3) return fail(LB_ENODATA, "fewer than 3 interface crossings in the window");
    // Normal equations of x^2 + y^2 + D x + E y + F = 0 in coordinates centred on the mean.
    double mx = 0, my = 0;
    for (size_t i = 0; i < m; ++i) { mx += px[i]; my += py[i]; }
    mx /= m; my /= m;
    double S[3][4] = {{0}};
    for (size_t i = 0; i < m; ++i) {
        const double a[3] = {px[i] - mx, py[i] - my, 1.0};
        const double z = -(a[0] * a[0] + a[1] * a[1]);
        for (int r = 0; r < 3; ++r) {
            for (int s = 0; s < 3; ++s) S[r][s] += a[r] * a[s];
            S[r][3] += a[r] * z;
        }
    }
    for (int col = 0; col < 3; ++col) {  // Gaussian elimination, partial pivoting
        int piv = col;
        for (int r = col + 1; r < 3; ++r) if (std::fabs(S[r][col]) > std::fabs(S[piv][col])) piv = r;
        if (S[piv][col] == 0.0) return fail(LB_ENODATA, "degenerate crossing set (collinear)");
        for (int s = 0; s < 4; ++s) std::swap(S[col][s], S[piv][s]);
        for (int r = 0; r < 3; ++r) {
            if (r == col) continue;
            const double fct = S[r][col] / S[col][col];
            for (int s = col; s < 4; ++s) S[r][s] -= fct * S[col][s];
        }
    }
    const double D = S[0][3] / S[0][0], E = S[1][3] / S[1][1], F = S[2][3] / S[2][2];
    const double xc = mx - D / 2, yc = my - E / 2;
    const double r2 = D * D / 4 + E * E / 4 - F;
    if (!(r2 > 0)) return fail(LB_ENODATA, "circle fit failed");
    const double R = std::sqrt(r2);
    if (xc_out) *xc_out = xc;
    if (yc_out) *yc_out = yc;
    if (r_out) *r_out = R;
    if (std::fabs(yc - y_wall) > R) return fail(LB_ENODATA, "fitted circle does not reach the wall");
    size_t inside = 0;
    for (size_t i = 0; i < m; ++i)
        if (std::hypot(ex[i] - xc, ey[i] - yc) < R) ++inside;
    double cosv = -wall_dir * (yc - y_wall) / R;
    cosv = std::max(-1.0, std::min(1.0, cosv));
    double th = std::acos(cosv) * 180.0 / M_PI;
    if (!(2 * inside > m)) th = 180.0 - th;
    *theta = th;
    return LB_OK;
}

int alloc_group_single(Group& g, const lb_params* p, void* ext, size_t ext_bytes) {
    g.m.resize(1);
    Member& mb = g.m[0];
    mb.L = make_layout(p->nx, p->ny, p->storage, p->inplace != 0);
    if (ext) {
        if (ext_bytes < mb.L.total) return fail(LB_ENOMEM, "device buffer smaller than lb_workspace_bytes");
        if (reinterpret_cast<uintptr_t>(ext) % 256) return fail(LB_EINVAL, "device buffer must be 256-byte aligned");
        mb.base = reinterpret_cast<char*>(ext);
    } else {
        hipError_t e = hipMalloc(&g.alloc, mb.L.total);
        if (e != hipSuccess) {
            g.alloc = nullptr;
            return fail(LB_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
        }
        mb.base = g.alloc;
    }
    return LB_OK;
}

void free_group(Group& g) {
    if (g.stream) (void)hipStreamSynchronize(g.stream);
    destroy_graphs(g);
    if (g.capture_stream) (void)hipStreamDestroy(g.capture_stream);
    if (g.alloc) (void)hipFree(g.alloc);
    if (g.batch_alloc) (void)hipFree(g.batch_alloc);
    g.alloc = nullptr;
    g.batch_alloc = nullptr;
}

int pick_default_tiling(Group& g);

int init_single(const lb_params* p, const uint8_t* solid, const double* dphi, const double* phi0,
                const double* rho0, const double* ux0, const double* uy0, void* stream, void* ext,
                size_t ext_bytes, lb_handle** out) {
    Range range("lb_init");
    if (!out) return fail(LB_EINVAL, "out is NULL");
    *out = nullptr;
    int rc = validate_params(p);
    if (rc) return rc;
    int64_t nf = 0;
    rc = validate_inputs(p, solid, dphi, phi0, rho0, ux0, uy0, &nf);
    if (rc) return rc;
    lb_handle* h = new lb_handle();
    Group& g = h->g;
    g.stream = reinterpret_cast<hipStream_t>(stream);
    g.block_x = 256;
    g.rows = 32;
    rc = alloc_group_single(g, p, ext, ext_bytes);
    if (!rc) rc = init_member(g.m[0], p, solid, dphi, phi0, rho0, ux0, uy0, g.stream);
    if (!rc) rc = pick_default_tiling(g);
    if (rc) {
        const std::string msg = g_err;
        free_group(g);
        delete h;
        return fail(rc, msg);
    }
    g.m[0].n_fluid = nf;
    // In place, S_0 is stored in the layout that phase 1 reads.
    g.parity = p->inplace ? 1 : 0;
    *out = h;
    return LB_OK;
}

// Save the state buffer, run `fn`, restore the state, step and parity.
template <class Fn>
int with_restored_state(Group& g, Fn fn) {
    std::vector<std::vector<char>> host;
    HIPCHK(hipStreamSynchronize(g.stream));
    for (auto& mb : g.m) {
        host.emplace_back(mb.L.buf_bytes);
        HIPCHK(hipMemcpy(host.back().data(), mb.view.buf[g.parity], mb.L.buf_bytes,
                         hipMemcpyDeviceToHost));
    }
    const int par = g.parity;
    const int64_t step = g.step;
    int rc = fn();
    HIPCHK(hipStreamSynchronize(g.stream));
    for (size_t k = 0; k < g.m.size(); ++k)
        HIPCHK(hipMemcpy(g.m[k].view.buf[par], host[k].data(), g.m[k].L.buf_bytes,
                         hipMemcpyHostToDevice));
    g.parity = par;
    g.step = step;
    return rc;
}

int set_tuning(Group& g, int bx, int rows) {
    int rc = check_tuning(bx, rows);
    if (rc) return rc;
    if (bx == 1024 && g.m[0].p.storage == LB_F64C)
        return fail(LB_EINVAL, "LB_F64C takes block_x up to 512");
    if (g.batched) {
        const int old_bx = g.block_x, old_rows = g.rows;
        g.block_x = bx;
        g.rows = rows;
        if (current_tiles(g) > g.n_tiles) {
            g.block_x = old_bx;
            g.rows = old_rows;
            return fail(LB_EINVAL, "tuning needs more tiles than were allocated");
        }
        destroy_graphs(g);
        int rc2 = build_tiles(g);
        if (rc2) return rc2;
        if (g.schedule == LB_SCHEDULE_PERSISTENT) {
            std::string why;
            if (!persistent_ok(g, &why)) {
                g.block_x = old_bx;
                g.rows = old_rows;
                rc2 = build_tiles(g);
                return rc2 ? rc2 : fail(LB_EINVAL, why);
            }
            rc2 = persistent_grid(g);
        }
        return rc2;
    }
    g.block_x = bx;
    g.rows = rows;
    destroy_graphs(g);
    return LB_OK;
}

int set_schedule(Group& g, int schedule) {
    if (schedule != LB_SCHEDULE_STEPWISE && schedule != LB_SCHEDULE_PERSISTENT)
        return fail(LB_EINVAL, "schedule must be LB_SCHEDULE_STEPWISE or LB_SCHEDULE_PERSISTENT");
    if (schedule == LB_SCHEDULE_PERSISTENT) {
        std::string why;
        if (!persistent_ok(g, &why)) return fail(LB_EINVAL, why);
        int rc = persistent_grid(g);
        if (rc) return rc;
    }
    if (schedule != g.schedule) destroy_graphs(g);
    g.schedule = schedule;
    return LB_OK;
}

std::mutex g_tune_mu;
// Keyed by the current device's architecture name as well as the problem, so
// one process driving devices of different kinds tunes each.
// The kernel variant is part of the problem: tau_phi = 1 selects its own sweep
// instance, lattice-node bounce-back adds the wall launch and the tau table
// changes the per-node arithmetic.
using TuneKey = std::tuple<std::string, int, int, int, int, int, int, int, int, int>;
std::map<TuneKey, std::tuple<int, int, int>> g_tune_cache;  // block_x, rows, schedule

TuneKey tune_key(const Group& g, const char* arch) {
    int max_ny = 0, total = 0, any_bounce = 0, any_lut = 0;
    for (auto& mb : g.m) {
        max_ny = std::max(max_ny, mb.p.ny);
        total += mb.p.nx * mb.p.ny;
        any_bounce |= mb.p.bounce == LB_LATTICE_NODE;
        any_lut |= mb.p.tau_lut > 1;
    }
    return TuneKey(std::string(arch), g.m[0].p.nx, max_ny, g.m[0].p.storage, g.m[0].p.collision,
                   g.m[0].p.inplace, g.batched ? total : -1, g.m[0].p.tau_phi == 1.0, any_bounce,
                   any_lut);
}

// Tile shape of a new single lattice: the autotuner's earlier choice for the
// same problem on this device if there is one; otherwise the tallest strips
// and widest tiles (from 256 x 32 down to 64 x 4) that still give at least one
// workgroup per CU, so that small lattices spread over the chip. A lattice
// whose step moves under 64 MB is bound by the latency of a strip's walk (a
// strip of r rows waits on r + 4 rows of loads in turn, about 1.7 us each),
// not by bandwidth, so it takes one-row strips at the widest tile that still
// gives a workgroup per CU (1.5-1.8x the 4-row rate on 5,000-65,000 nodes).
int pick_default_tiling(Group& g) {
    int dev = 0, cus = 0;
    hipDeviceProp_t prop;
    HIPCHK(hipGetDevice(&dev));
    HIPCHK(hipGetDeviceProperties(&prop, dev));
    HIPCHK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune_cache.find(tune_key(g, prop.gcnArchName));
        if (it != g_tune_cache.end()) {
            g.block_x = std::get<0>(it->second);
            g.rows = std::get<1>(it->second);
            return LB_OK;
        }
    }
    const int64_t nx = g.m[0].p.nx, ny = g.m[0].p.ny;
    const int st = g.m[0].p.storage;
    const int64_t lu_bytes = st == LB_F64 ? 288 : st == LB_F32 ? 144 : st == LB_F64C ? 208
                             : st == LB_F32C ? 104 : 88;
    const bool latency_bound = nx * ny * lu_bytes < (int64_t)64 << 20;
    g.block_x = 64;
    g.rows = latency_bound ? 1 : 4;
    for (int bx : {256, 128, 64})
        for (int rows : {32, 16, 8, 4}) {
            const int r = latency_bound ? 1 : rows;
            if (((nx + bx - 1) / bx) * ((ny + r - 1) / r) >= cus) {
                g.block_x = bx;
                g.rows = r;
                return LB_OK;
            }
        }
    return LB_OK;
}

int autotune(Group& g, int steps, lb_tuning* chosen) {
    Range range("lb autotune");
    if (steps < 1) return fail(LB_EINVAL, "steps_per_trial must be >= 1");
    int dev = 0;
    hipDeviceProp_t prop;
    HIPCHK(hipGetDevice(&dev));
    HIPCHK(hipGetDeviceProperties(&prop, dev));
    int max_ny = 0;
    for (auto& mb : g.m) max_ny = std::max(max_ny, mb.p.ny);
    const TuneKey key = tune_key(g, prop.gcnArchName);
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune_cache.find(key);
        if (it != g_tune_cache.end()) {
            int rc = set_schedule(g, LB_SCHEDULE_STEPWISE);
            if (!rc) rc = set_tuning(g, std::get<0>(it->second), std::get<1>(it->second));
            if (!rc) rc = set_schedule(g, std::get<2>(it->second));
            if (chosen) *chosen = lb_tuning{g.block_x, g.rows};
            return rc;
        }
    }
    // Candidates: (schedule, block_x, rows). Batches also try the persistent
    // schedule, with the strip heights scaled per member (member_rows).
    std::vector<std::tuple<int, int, int>> cands;
    for (int bx : {64, 128, 256, 512, 1024})
        for (int rows : {1, 2, 4, 8, 16, 32, 64, 128})
            cands.emplace_back(LB_SCHEDULE_STEPWISE, bx, rows);
    if (g.batched)
        for (int bx : {128, 256, 512})
            for (int rows : {4, 8, 16, 32}) cands.emplace_back(LB_SCHEDULE_PERSISTENT, bx, rows);
    const int sched_save = g.schedule;
    int best_bx = g.block_x, best_rows = g.rows, best_sched = g.schedule;
    float best = 1e30f;
    const int diag_save = g.m[0].p.diag_every;
    // Destroys the timing events on every return path of the trial loop.
    struct Events {
        hipEvent_t e0 = nullptr, e1 = nullptr;
        ~Events() {
            if (e0) (void)hipEventDestroy(e0);
            if (e1) (void)hipEventDestroy(e1);
        }
    };
    int rc = with_restored_state(g, [&]() -> int {
        for (auto& mb : g.m) mb.p.diag_every = 0;
        Events ev;
        HIPCHK(hipEventCreate(&ev.e0));
        HIPCHK(hipEventCreate(&ev.e1));
        hipEvent_t e0 = ev.e0, e1 = ev.e1;
        for (const auto& c : cands) {
            const int sched = std::get<0>(c), bx = std::get<1>(c), rows = std::get<2>(c);
            if (rows > 2 * max_ny) continue;
            if (set_schedule(g, LB_SCHEDULE_STEPWISE) || set_tuning(g, bx, rows) ||
                set_schedule(g, sched))
                continue;
            // Timed as the steps run: replays of one captured graph of `len`
            // steps (an even count, so each replay starts at the same parity),
            // after one untimed replay; the capture is not timed.
            int len = 2;
            while (len * 2 <= std::min(steps, kGraphSteps)) len *= 2;
            const int reps = (steps + len - 1) / len;
            hipGraphExec_t ge = nullptr;
            int crc = capture_graph(g, len, g.parity, false, &ge);
            if (crc) return crc;
            struct ExecGuard {
                hipGraphExec_t e;
                ~ExecGuard() { (void)hipGraphExecDestroy(e); }
            } guard{ge};
            HIPCHK(hipGraphLaunch(ge, g.stream));
            HIPCHK(hipEventRecord(e0, g.stream));
            for (int r = 0; r < reps; ++r) HIPCHK(hipGraphLaunch(ge, g.stream));
            HIPCHK(hipEventRecord(e1, g.stream));
            HIPCHK(hipEventSynchronize(e1));
            float ms = 0;
            HIPCHK(hipEventElapsedTime(&ms, e0, e1));
            ms /= (float)(reps * len);  // per step
            if (ms < best) {
                best = ms;
                best_bx = bx;
                best_rows = rows;
                best_sched = sched;
            }
        }
        return LB_OK;
    });
    for (auto& mb : g.m) mb.p.diag_every = diag_save;
    if (rc) {
        (void)set_schedule(g, sched_save);
        return rc;
    }
    rc = set_schedule(g, LB_SCHEDULE_STEPWISE);
    if (!rc) rc = set_tuning(g, best_bx, best_rows);
    if (!rc) rc = set_schedule(g, best_sched);
    if (rc) return rc;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tune_cache[key] = std::make_tuple(best_bx, best_rows, best_sched);
    }
    if (chosen) *chosen = lb_tuning{g.block_x, g.rows};
    return LB_OK;
}

// Parameters that define the computation, compared field by field (a struct
// compare would also compare padding bytes); diag_every may differ.
bool same_params(const lb_params& a, const lb_params& b) {
    return a.nx == b.nx && a.ny == b.ny && a.A == b.A && a.B == b.B && a.kappa == b.kappa &&
           a.Gamma == b.Gamma && a.tau_alpha == b.tau_alpha && a.tau_beta == b.tau_beta &&
           a.tau_phi == b.tau_phi && a.rho_ref == b.rho_ref && a.collision == b.collision &&
           a.storage == b.storage && a.zero_u_feq == b.zero_u_feq &&
           a.zero_u_geq == b.zero_u_geq && a.tau_clamp == b.tau_clamp &&
           a.inplace == b.inplace && a.tau_lut == b.tau_lut && a.bounce == b.bounce;
}

struct CkptHeader {
    char magic[8];
    int32_t version;
    int32_t parity;
    int64_t step;
    lb_params params;
    uint64_t buf_bytes;
    uint64_t n;
};

}  // namespace

// ======================================================================= C ABI

extern "C" {

const char* lb_last_error(void) { return g_err.c_str(); }

int lb_default_params(int32_t nx, int32_t ny, lb_params* p) {
    if (!p) return fail(LB_EINVAL, "params is NULL");
    *p = lb_params{};
    p->nx = nx;
    p->ny = ny;
    p->A = -0.04;
    p->B = 0.04;
    p->kappa = 0.04;
    p->Gamma = 0.1;
    p->tau_alpha = 1.0;
    p->tau_beta = 1.0;
    p->tau_phi = 1.0;
    p->rho_ref = 1.0;
    p->collision = LB_BGK;
    p->storage = LB_F64;
    return LB_OK;
}

int lb_workspace_bytes(const lb_params* p, size_t* bytes) {
    int rc = validate_params(p);
    if (rc) return rc;
    if (!bytes) return fail(LB_EINVAL, "bytes is NULL");
    *bytes = make_layout(p->nx, p->ny, p->storage, p->inplace != 0).total;
    return LB_OK;
}

int lb_init(const lb_params* p, const uint8_t* solid, const double* wall_dphi, const double* phi0,
            const double* rho0, const double* ux0, const double* uy0, void* stream,
            lb_handle** out) {
    return init_single(p, solid, wall_dphi, phi0, rho0, ux0, uy0, stream, nullptr, 0, out);
}

int lb_init_ext(const lb_params* p, const uint8_t* solid, const double* wall_dphi,
                const double* phi0, const double* rho0, const double* ux0, const double* uy0,
                void* stream, void* device_buffer, size_t buffer_bytes, lb_handle** out) {
    if (!device_buffer) return fail(LB_EINVAL, "device_buffer is NULL");
    return init_single(p, solid, wall_dphi, phi0, rho0, ux0, uy0, stream, device_buffer,
                       buffer_bytes, out);
}

int lb_step(lb_handle* h, int64_t nsteps) {
    Range r("lb_step");
    if (!h) return fail(LB_EINVAL, "handle is NULL");
    return group_step(h->g, nsteps);
}

int lb_get_step(lb_handle* h, int64_t* step) {
    if (!h || !step) return fail(LB_EINVAL, "NULL argument");
    *step = h->g.step;
    return LB_OK;
}

int lb_read_fields(lb_handle* h, double* phi, double* rho, double* ux, double* uy) {
    if (!h) return fail(LB_EINVAL, "handle is NULL");
    int rc = read_fields(h->g, 0, phi, rho, ux, uy);
    if (rc) return rc;
    return check_flag(h->g);
}

int lb_read_populations(lb_handle* h, double* f, double* g) {
    if (!h) return fail(LB_EINVAL, "handle is NULL");
    return read_populations(h->g, 0, f, g);
}

int lb_diagnostics(lb_handle* h, lb_diag* d) {
    if (!h || !d) return fail(LB_EINVAL, "NULL argument");
    double s[6];
    int rc = reduce_member(h->g, 0, 0, 0, s);
    if (rc) return rc;
    d->sum_rho = s[0];
    d->sum_phi = s[1];
    d->kinetic = s[2];
    d->max_u = s[3];
    d->n_fluid = (int64_t)std::llround(s[4]);
    d->step = h->g.step;
    if (!is_finite(s[0]) || !is_finite(s[1]) || !is_finite(s[2]) || !(s[3] == s[3]))
        return fail(LB_ENUMERIC, "non-finite conservation sums");
    return check_flag(h->g);
}

int lb_diagnostics_noalloc(lb_handle* h, lb_diag* d) {
    if (!h || !d) return fail(LB_EINVAL, "NULL argument");
    Group& g = h->g;
    Member& mb = g.m[0];
    const int64_t n = (int64_t)mb.p.nx * mb.p.ny;
    const int64_t nrec = (n + 255) / 256;
    if (nrec > (int64_t)kScratchRecords)
        return fail(LB_EINVAL, "lb_diagnostics_noalloc takes lattices of at most 2^23 nodes "
                               "(its scratch holds 2^15 partial records of 256 nodes)");
    void* base = nullptr;
    int rc = scratch_address(&base);
    if (rc) return rc;
    double* partials = reinterpret_cast<double*>(base);
    double* rec_dev = partials + kScratchRecords * kPartials;
    int32_t* flag = reinterpret_cast<int32_t*>(rec_dev + kPartials);
    // The array keeps the last call's contents: the flag word must start at
    // zero (a fill kernel, so the call can also sit inside a captured graph);
    // the partial records and the finished record are written in full below.
    HIPCHK(launch_fill(flag, 0, 4, g.stream));
    HIPCHK(launch_moments(mb.view, g.parity, 0, n, nullptr, partials, (int)kScratchRecords, 0, 0,
                          g.stream));
    HIPCHK(launch_finalize(nullptr, nullptr, 1, (int)nrec, partials, rec_dev, flag, g.stream));
    double rec[kPartials];
    HIPCHK(hipMemcpyAsync(rec, rec_dev, sizeof(rec), hipMemcpyDeviceToHost, g.stream));
    HIPCHK(hipStreamSynchronize(g.stream));
    d->sum_rho = rec[0];
    d->sum_phi = rec[1];
    d->kinetic = rec[2];
    d->max_u = rec[3];
    d->n_fluid = (int64_t)std::llround(rec[4]);
    d->step = g.step;
    if (!is_finite(rec[0]) || !is_finite(rec[1]) || !is_finite(rec[2]) || !(rec[3] == rec[3]))
        return fail(LB_ENUMERIC, "non-finite conservation sums");
    return check_flag(g);
}

int lb_contact_angle(lb_handle* h, double x_lo, double x_hi, double y_lo, double y_hi,
                     double y_wall, int32_t wall_dir, double* theta_deg, double* xc, double* yc,
                     double* radius, int64_t* n_points) {
    if (!h) return fail(LB_EINVAL, "handle is NULL");
    return contact_angle(h->g, 0, x_lo, x_hi, y_lo, y_hi, y_wall, wall_dir, theta_deg, xc, yc,
                         radius, n_points);
}

int lb_fill_length(lb_handle* h, int32_t x_lo, int32_t x_hi, double width, double* length) {
    if (!h || !length) return fail(LB_EINVAL, "NULL argument");
    if (!(width > 0)) return fail(LB_EINVAL, "width must be positive");
    if (x_hi < x_lo) return fail(LB_EINVAL, "x_hi < x_lo");
    double s[6];
    int rc = reduce_member(h->g, 0, x_lo, x_hi, s);
    if (rc) return rc;
    *length = s[5] / width;
    return LB_OK;
}

int lb_set_wall_dphi(lb_handle* h, const double* wall_dphi) {
    if (!h) return fail(LB_EINVAL, "handle is NULL");
    Member& mb = h->g.m[0];
    const int64_t n = (int64_t)mb.p.nx * mb.p.ny;
    if (wall_dphi)
        for (int64_t i = 0; i < n; ++i)
            if (mb.solid[i] && !is_finite(wall_dphi[i])) return fail(LB_EINVAL, "non-finite wall_dphi");
    HIPCHK(hipStreamSynchronize(h->g.stream));
    return upload_dphi(mb, wall_dphi, h->g.stream);
}

int lb_save(lb_handle* h, const char* path) {
    if (!h || !path) return fail(LB_EINVAL, "NULL argument");
    Group& g = h->g;
    Member& mb = g.m[0];
    HIPCHK(hipStreamSynchronize(g.stream));
    std::vector<char> buf(mb.L.buf_bytes);
    HIPCHK(hipMemcpy(buf.data(), mb.view.buf[g.parity], buf.size(), hipMemcpyDeviceToHost));
    CkptHeader hd{};
    std::memcpy(hd.magic, "LBMCKPT1", 8);
    hd.version = 1;
    // In place, the layout of the state depends on the phase.
    hd.parity = mb.p.inplace ? g.parity : 0;
    hd.step = g.step;
    hd.params = mb.p;
    hd.buf_bytes = buf.size();
    hd.n = (uint64_t)mb.p.nx * mb.p.ny;
    FILE* fp = std::fopen(path, "wb");
    if (!fp) return fail(LB_EIO, std::string("cannot open ") + path);
    bool ok = std::fwrite(&hd, sizeof(hd), 1, fp) == 1 &&
              std::fwrite(mb.solid.data(), 1, hd.n, fp) == hd.n &&
              std::fwrite(mb.dphi.data(), 8, hd.n, fp) == hd.n &&
              std::fwrite(buf.data(), 1, buf.size(), fp) == buf.size();
    ok = (std::fclose(fp) == 0) && ok;
    if (!ok) return fail(LB_EIO, std::string("write failed: ") + path);
    return LB_OK;
}

int lb_load(lb_handle* h, const char* path) {
    if (!h || !path) return fail(LB_EINVAL, "NULL argument");
    Group& g = h->g;
    Member& mb = g.m[0];
    FILE* fp = std::fopen(path, "rb");
    if (!fp) return fail(LB_EIO, std::string("cannot open ") + path);
    CkptHeader hd{};
    std::vector<uint8_t> solid;
    std::vector<double> dphi;
    std::vector<char> buf;
    bool ok = std::fread(&hd, sizeof(hd), 1, fp) == 1 && std::memcmp(hd.magic, "LBMCKPT1", 8) == 0 &&
              hd.version == 1 && hd.n == (uint64_t)mb.p.nx * mb.p.ny && hd.buf_bytes == mb.L.buf_bytes &&
              (hd.parity == 0 || (hd.parity == 1 && mb.p.inplace));
    if (ok) {
        solid.resize(hd.n);
        dphi.resize(hd.n);
        buf.resize(hd.buf_bytes);
        ok = std::fread(solid.data(), 1, hd.n, fp) == hd.n &&
             std::fread(dphi.data(), 8, hd.n, fp) == hd.n &&
             std::fread(buf.data(), 1, buf.size(), fp) == buf.size();
    }
    std::fclose(fp);
    if (!ok) return fail(LB_EIO, std::string("not a matching checkpoint: ") + path);
    if (!same_params(hd.params, mb.p) || solid != mb.solid)
        return fail(LB_EINVAL, "checkpoint parameters or mask differ from the handle");
    HIPCHK(hipStreamSynchronize(g.stream));
    HIPCHK(hipMemcpy(mb.view.buf[0], buf.data(), buf.size(), hipMemcpyHostToDevice));
    // The loaded state replaces whatever the periodic check saw before: clear
    // the sticky non-finite flag (and its scratch neighbour).
    HIPCHK(launch_fill(mb.base + mb.L.off_flag, 0, 8, g.stream));
    g.parity = hd.parity;
    g.step = hd.step;
    return upload_dphi(mb, dphi.data(), g.stream);
}

int lb_set_tuning(lb_handle* h, const lb_tuning* t) {
    if (!h || !t) return fail(LB_EINVAL, "NULL argument");
    HIPCHK(hipStreamSynchronize(h->g.stream));
    return set_tuning(h->g, t->block_x, t->rows_per_block);
}

int lb_get_tuning(lb_handle* h, lb_tuning* t) {
    if (!h || !t) return fail(LB_EINVAL, "NULL argument");
    *t = lb_tuning{h->g.block_x, h->g.rows};
    return LB_OK;
}

int lb_autotune(lb_handle* h, int32_t steps_per_trial, lb_tuning* chosen) {
    if (!h) return fail(LB_EINVAL, "handle is NULL");
    return autotune(h->g, steps_per_trial, chosen);
}

int lb_free(lb_handle* h) {
    if (!h) return LB_OK;
    free_group(h->g);
    delete h;
    return LB_OK;
}

int lb_dphi_for_angle(double theta_deg, double kappa, double A, double B, double* dphi) {
    if (!dphi) return fail(LB_EINVAL, "dphi is NULL");
    if (!(theta_deg >= 0.0 && theta_deg <= 180.0)) return fail(LB_EINVAL, "theta must be in [0, 180]");
    if (!(kappa > 0) || !(B > 0) || !(A < 0)) return fail(LB_EINVAL, "need kappa > 0, B > 0, A < 0");
    // The closed form assumes the symmetric double well B = -A = a.
    if (std::fabs(A + B) > 1e-12 * B) return fail(LB_EINVAL, "closed form needs B == -A");
    const double a = B;
    const double th = theta_deg * M_PI / 180.0;
    const double s = std::sin(th);
    const double alpha = std::acos(s * s);
    const double c3 = std::cos(alpha / 3.0);
    const double sg = th > M_PI / 2 ? 1.0 : (th < M_PI / 2 ? -1.0 : 0.0);
    *dphi = 2.0 * sg * std::sqrt(std::max(0.0, c3 * (1.0 - c3))) / std::sqrt(2.0 * kappa / a);
    return LB_OK;
}

int lb_bandwidth_probe(size_t bytes, int32_t repeats, void* stream, double* gbs) {
    if (!gbs || repeats < 1 || bytes < (1u << 20)) return fail(LB_EINVAL, "need bytes >= 1 MiB, repeats >= 1");
    bytes &= ~(size_t)255;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    char* a = nullptr;
    char* b = nullptr;
    if (hipMalloc(&a, bytes) != hipSuccess) return fail(LB_ENOMEM, "probe allocation failed");
    if (hipMalloc(&b, bytes) != hipSuccess) {
        (void)hipFree(a);
        return fail(LB_ENOMEM, "probe allocation failed");
    }
    int rc = LB_OK;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    do {
        int dev = 0, cus = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
            rc = fail(LB_EHIP, "device query failed");
            break;
        }
        if (launch_fill(a, 1, bytes, st) != hipSuccess || hipEventCreate(&e0) != hipSuccess ||
            hipEventCreate(&e1) != hipSuccess) {
            rc = fail(LB_EHIP, "probe launch failed");
            break;
        }
        // Three copy kernels at four grid sizes (workgroups per CU); the best rate.
        double best = 0.0;
        for (int cfg = 0; cfg < 12 && rc == LB_OK; ++cfg) {
            const int variant = cfg / 4, blocks = cus * (2 << (cfg % 4));
            if (launch_stream_copy(a, b, bytes, blocks, variant, st) != hipSuccess ||
                hipEventRecord(e0, st) != hipSuccess) {
                rc = fail(LB_EHIP, "probe launch failed");
                break;
            }
            for (int r = 0; r < repeats && rc == LB_OK; ++r)
                if (launch_stream_copy(a, b, bytes, blocks, variant, st) != hipSuccess)
                    rc = fail(LB_EHIP, "probe launch failed");
            float ms = 0;
            if (rc == LB_OK && (hipEventRecord(e1, st) != hipSuccess ||
                                hipEventSynchronize(e1) != hipSuccess ||
                                hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
                rc = fail(LB_EHIP, "probe timing failed");
            if (rc != LB_OK) break;
            best = std::max(best, 2.0 * (double)bytes * repeats / (ms * 1e-3) / 1e9);
        }
        if (rc == LB_OK) *gbs = best;
    } while (0);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFree(a);
    (void)hipFree(b);
    return rc;
}

// ---------------------------------------------------------------- batches

int lb_batch_init(int32_t n, const lb_params* params, const uint8_t* const* solid,
                  const double* const* wall_dphi, const double* const* phi0,
                  const double* const* rho0, const double* const* ux0, const double* const* uy0,
                  void* stream, const lb_tuning* tuning, lb_batch** out) {
    Range range("lb_batch_init");
    if (!out) return fail(LB_EINVAL, "out is NULL");
    *out = nullptr;
    if (n < 1 || !params || !solid || !phi0) return fail(LB_EINVAL, "need n >= 1, params, solid, phi0");
    std::vector<int64_t> nf(n);
    for (int k = 0; k < n; ++k) {
        int rc = validate_params(&params[k]);
        if (!rc)
            rc = validate_inputs(&params[k], solid[k], wall_dphi ? wall_dphi[k] : nullptr, phi0[k],
                                 rho0 ? rho0[k] : nullptr, ux0 ? ux0[k] : nullptr,
                                 uy0 ? uy0[k] : nullptr, &nf[k]);
        if (rc) return fail(rc, "member " + std::to_string(k) + ": " + g_err);
        if (params[k].inplace)
            return fail(LB_EINVAL, "member " + std::to_string(k) +
                                       ": in-place update is for single lattices (lb_init)");
        if (params[k].storage != params[0].storage || params[k].collision != params[0].collision ||
            params[k].zero_u_feq != params[0].zero_u_feq ||
            params[k].zero_u_geq != params[0].zero_u_geq ||
            params[k].diag_every != params[0].diag_every ||
            (params[k].tau_phi == 1.0) != (params[0].tau_phi == 1.0))
            return fail(LB_EINVAL,
                        "members must share storage, collision, Step 2 flags, diag_every and "
                        "whether tau_phi is 1");
    }
    int bx = 256, rows = 32;
    if (tuning) {
        int rc = check_tuning(tuning->block_x, tuning->rows_per_block);
        if (rc) return rc;
        bx = tuning->block_x;
        rows = tuning->rows_per_block;
    }
    lb_batch* b = new lb_batch();
    Group& g = b->g;
    g.batched = true;
    for (int k = 0; k < n; ++k)
        if (params[k].bounce == LB_LATTICE_NODE) g.any_walls = true;
    g.stream = reinterpret_cast<hipStream_t>(stream);
    g.block_x = bx;
    g.rows = rows;
    g.m.resize(n);
    size_t total = 0;
    size_t tiles_max = 0;
    std::vector<size_t> offs(n);
    for (int k = 0; k < n; ++k) {
        g.m[k].L = make_layout(params[k].nx, params[k].ny, params[k].storage, false);
        offs[k] = total;
        total += round_up(g.m[k].L.total, 256);
        tiles_max += g.m[k].L.n_tiles_max;
    }
    g.n_tiles = (int)tiles_max;
    // The stepwise table pads the XCDs' lists to one length: at most 8 entries
    // per logical tile.
    g.step_slots_max = (int)(8 * tiles_max);
    const size_t off_tiles = total;
    const size_t off_first = off_tiles + round_up(8 * tiles_max * sizeof(Tile), 256);
    const size_t off_part = off_first + round_up((size_t)(n + 1) * 4, 256);
    const size_t off_diag = off_part + round_up(tiles_max * kPartials * 8, 256);
    const size_t off_flag = off_diag + round_up((size_t)n * kPartials * 8, 256);
    const size_t off_views = off_flag + round_up((size_t)n * 4, 256);
    const size_t off_ptiles = off_views + round_up((size_t)n * sizeof(View), 256);
    const size_t off_deps = off_ptiles + round_up(tiles_max * sizeof(Tile), 256);
    const size_t off_sync = off_deps + round_up(tiles_max * kPersistDeps * 4, 256);
    const size_t bytes = off_sync + round_up((tiles_max + 2) * 4, 256);
    hipError_t e = hipMalloc(&g.batch_alloc, bytes);
    if (e != hipSuccess) {
        g.batch_alloc = nullptr;
        delete b;
        return fail(LB_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
    }
    char* base = g.batch_alloc;
    g.d_tiles = reinterpret_cast<Tile*>(base + off_tiles);
    g.d_first = reinterpret_cast<int32_t*>(base + off_first);
    g.d_partials = reinterpret_cast<double*>(base + off_part);
    g.d_diag = reinterpret_cast<double*>(base + off_diag);
    g.d_flag = reinterpret_cast<int32_t*>(base + off_flag);
    g.d_views = reinterpret_cast<View*>(base + off_views);
    g.d_ptiles = reinterpret_cast<Tile*>(base + off_ptiles);
    g.d_deps = reinterpret_cast<int32_t*>(base + off_deps);
    g.d_sync = reinterpret_cast<int32_t*>(base + off_sync);
    int rc = LB_OK;
    if (launch_fill(base + off_tiles, 0, bytes - off_tiles, g.stream) != hipSuccess)
        rc = fail(LB_EHIP, "fill failed");
    std::vector<View> views(n);
    for (int k = 0; k < n && !rc; ++k) {
        g.m[k].base = base + offs[k];
        rc = init_member(g.m[k], &params[k], solid[k], wall_dphi ? wall_dphi[k] : nullptr, phi0[k],
                         rho0 ? rho0[k] : nullptr, ux0 ? ux0[k] : nullptr, uy0 ? uy0[k] : nullptr,
                         g.stream);
        g.m[k].n_fluid = nf[k];
        views[k] = g.m[k].view;
    }
    if (!rc && hipMemcpy(g.d_views, views.data(), n * sizeof(View), hipMemcpyHostToDevice) != hipSuccess)
        rc = fail(LB_EHIP, "copy of member views failed");
    if (!rc) rc = build_tiles(g);
    // No tuning given: time the candidate tile shapes on the ensemble itself
    // (state restored afterwards, so results do not depend on the choice).
    if (!rc && !tuning) rc = autotune(g, kBatchTuneSteps, nullptr);
    if (rc) {
        const std::string msg = g_err;
        free_group(g);
        delete b;
        return fail(rc, msg);
    }
    *out = b;
    return LB_OK;
}

int lb_batch_step(lb_batch* b, int64_t nsteps) {
    Range r("lb_batch_step");
    if (!b) return fail(LB_EINVAL, "batch is NULL");
    return group_step(b->g, nsteps);
}

static int check_member(lb_batch* b, int32_t k) {
    if (!b) return fail(LB_EINVAL, "batch is NULL");
    if (k < 0 || k >= (int32_t)b->g.m.size()) return fail(LB_EINVAL, "member index out of range");
    return LB_OK;
}

int lb_batch_read_fields(lb_batch* b, int32_t k, double* phi, double* rho, double* ux, double* uy) {
    int rc = check_member(b, k);
    if (rc) return rc;
    rc = read_fields(b->g, k, phi, rho, ux, uy);
    if (rc) return rc;
    return check_flag(b->g);
}

int lb_batch_read_populations(lb_batch* b, int32_t k, double* f, double* g) {
    int rc = check_member(b, k);
    if (rc) return rc;
    rc = check_windows(b->g);
    if (rc) return rc;
    return read_populations(b->g, k, f, g);
}

int lb_batch_contact_angle(lb_batch* b, int32_t k, double x_lo, double x_hi, double y_lo,
                           double y_hi, double y_wall, int32_t wall_dir, double* theta_deg) {
    int rc = check_member(b, k);
    if (rc) return rc;
    rc = check_windows(b->g);
    if (rc) return rc;
    return contact_angle(b->g, k, x_lo, x_hi, y_lo, y_hi, y_wall, wall_dir, theta_deg, nullptr,
                         nullptr, nullptr, nullptr);
}

int lb_batch_autotune(lb_batch* b, int32_t steps_per_trial, lb_tuning* chosen) {
    if (!b) return fail(LB_EINVAL, "batch is NULL");
    return autotune(b->g, steps_per_trial, chosen);
}

int lb_batch_set_schedule(lb_batch* b, int32_t schedule, uint32_t spin_limit) {
    if (!b) return fail(LB_EINVAL, "batch is NULL");
    HIPCHK(hipStreamSynchronize(b->g.stream));
    int rc = set_schedule(b->g, schedule);
    if (rc) return rc;
    b->g.spin_limit = spin_limit ? spin_limit : kDefaultSpinLimit;
    destroy_graphs(b->g);  // the poll limit is a launch argument
    return LB_OK;
}

int lb_batch_get_schedule(lb_batch* b, int32_t* schedule) {
    if (!b || !schedule) return fail(LB_EINVAL, "NULL argument");
    *schedule = b->g.schedule;
    return LB_OK;
}

int lb_batch_get_tuning(lb_batch* b, lb_tuning* t) {
    if (!b || !t) return fail(LB_EINVAL, "NULL argument");
    *t = lb_tuning{b->g.block_x, b->g.rows};
    return LB_OK;
}

int lb_batch_free(lb_batch* b) {
    if (!b) return LB_OK;
    free_group(b->g);
    delete b;
    return LB_OK;
}

}  // extern "C"
