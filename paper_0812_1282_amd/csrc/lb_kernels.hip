// HIP kernels for gfx950 of the binary free-energy lattice Boltzmann method of
// Pooley, Kusumaatmaja and Yeomans (arXiv:0812.1282).
//
// The hot path is sweep_kernel: one fused pass per timestep (pull-stream with
// mid-link bounce-back, moments, LDS phi tile with wetting ghosts, stencils,
// mu and p0, tau(phi), equilibria, BGK or MRT collision, store). It is bound by
// HBM bandwidth: every population is read once and written once per step.
//
// Work decomposition: a workgroup of BX threads owns BX consecutive columns
// (one per thread, coalesced along x) and walks `rows` consecutive rows of a
// strip. phi of the rows it needs is kept in an 8-row ring in LDS, two rows
// ahead of the row being collided, with two halo columns on each side; the
// pulled g of the two look-ahead rows stays in registers, so every g value is
// loaded once for phi and reused by the collision.
//
// Addressing: for a row, every plane's row start is uniform across the
// workgroup (kept in scalar registers) and each lane adds a 32-bit byte offset
// for its column, so loads and stores use the global "scalar base + vector
// offset" form. Bounce-back is a per-node fix-up after the regular pulls (only
// nodes next to a wall take it).
//
// Arithmetic: FP64 for the FP64 format. The other formats store f_i - r_i, r_i
// the rest state of a bulk phase at rho_ref, and do the FP32 arithmetic on
// those deviations (rho - rho_ref, p0 - p0(rest), f^eq - r), which keeps the
// small pressure differences that drive the interface (gamma / R) well above
// FP32 rounding of O(1) quantities.
#include "lb_internal.h"

#include <hip/hip_runtime.h>
#include <math.h>

#include <type_traits>

#define GLOBAL __attribute__((address_space(1)))

namespace lbm {

// D2Q9 vectors of Sec. III.A and their opposites.
__device__ constexpr int EX[9] = {0, 1, -1, 0, 0, 1, -1, -1, 1};
__device__ constexpr int EY[9] = {0, 0, 0, 1, -1, 1, -1, 1, -1};
__device__ constexpr int OPP[9] = {0, 2, 1, 4, 3, 6, 5, 8, 7};

// ------------------------------------------------------------------ storage

__device__ inline float bf16_to_float(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }
// Round to nearest even; gfx950 converts in one instruction (v_cvt_pk_bf16_f32).
__device__ inline uint16_t float_to_bf16(float f) { return __builtin_bit_cast(uint16_t, (__bf16)f); }

// Storage format traits. Plane p: 0..8 = f_0..f_8, 9..17 = g_0..g_8.
//   E<p>    element type of plane p
//   dec/enc conversion between a stored element and the working value
// Working values of f planes are deviations f_i - r_i in the shifted formats.
// The 16-bit formats keep the f_2, f_4..f_8 deviations times 2^6 and g_1..g_8
// times 2^10, so that the small values stay out of the FP16 subnormal range
// (powers of two: the scaling itself is exact); the f_0, f_1, f_3 deviations
// and g_0 are 32-bit, so that the stored set of a node can carry its mass and
// momentum exactly (see the store in the sweep).
template <int S>
struct Fmt;

// g_0 in the shifted formats. g_0 is close to phi, i.e. to +-1 in a bulk phase,
// where FP32 resolves only 6e-8: rounding it every step would create or destroy
// phi at each node. It is therefore kept as g_0 = b + q with b in {-1, 0, 1}
// and q small: q is an FP32 value rounded to nearest-even at 21 bits whose two
// lowest significand bits hold b + 1. The sweep keeps b and the small sums
// apart, so the stored g of a node add up to its phi to about 1e-9.
struct G0Code {
    __device__ static float q(uint32_t u) { return __builtin_bit_cast(float, u & ~3u); }
    __device__ static float b(uint32_t u) { return (float)((int)(u & 3u) - 1); }
    __device__ static uint32_t enc(float q, float b) {
        const uint32_t u = __builtin_bit_cast(uint32_t, q);
        return ((u + 1u + ((u >> 2) & 1u)) & ~3u) | (uint32_t)((int)b + 1);
    }
    // Keep b while |q| <= 3/4 (no switching back and forth for a node at
    // g_0 ~ +-1/2), else move b to the value nearest b + q.
    template <class T>
    __device__ static void rebase(T& q, T& b) {
        if (q > (T)0.75 || q < (T)-0.75) {
            const T t = b + q;
            const T nb = t > (T)0.5 ? (T)1 : (t < (T)-0.5 ? (T)-1 : (T)0);
            q += b - nb;
            b = nb;
        }
    }
};

template <>
struct Fmt<ST_F64> {
    using real = double;
    static constexpr bool shifted = false;
    static constexpr bool gstate = false;
    static constexpr bool packed = false;
    template <int p>
    static constexpr uint32_t colmul() { return 1; }
    template <int p> using E = double;
    template <int p>
    __device__ static int poff(const View& v) { return p * v.pitch * 8; }
    template <int p>
    __device__ static real dec(double x) { return x; }
    template <int p>
    __device__ static double enc(real x) { return x; }
};

#ifndef LB_F32_REAL
#define LB_F32_REAL float
#endif
template <>
struct Fmt<ST_F32> {
    using real = LB_F32_REAL;
    static constexpr bool shifted = true;
    static constexpr bool gstate = false;
    static constexpr bool packed = false;
    template <int p>
    static constexpr uint32_t colmul() { return 1; }
    template <int p> using E = typename std::conditional<p == 9, uint32_t, float>::type;
    template <int p>
    __device__ static int poff(const View& v) { return p * v.pitch * 4; }
    template <int p>
    __device__ static real dec(E<p> x) {
        static_assert(p != 9, "g_0 goes through G0Code");
        return x;
    }
    template <int p>
    __device__ static E<p> enc(real x) {
        static_assert(p != 9, "g_0 goes through G0Code");
        return x;
    }
};

template <int S>
struct Fmt16 {
    using real = float;
    static constexpr bool shifted = true;
    static constexpr bool gstate = false;
    static constexpr float kF = 64.0f, kG = 1024.0f;
    // f_i and g_i for i = 2, 4..8 are pulled from the same node (or bounce back
    // together), so they share one 32-bit word: f in the low half, g in the
    // high half. One load or store then moves both.
    static constexpr bool packed = true;
    static constexpr bool paired(int i) { return i == 2 || (i >= 4 && i <= 8); }
    static constexpr bool wide(int p) { return p == 0 || p == 1 || p == 3; }
    template <int p>
    using E = typename std::conditional<
        p == 9, uint32_t, typename std::conditional<wide(p), float, uint16_t>::type>::type;
    // Row block (pitch P): the pair words of i = 2, 4, 5, 6, 7, 8 (4P bytes
    // each), g_1 and g_3 (16-bit, 2P each), then f_1, f_3, f_0 and g_0 (32-bit).
    static constexpr int pair_slot(int i) { return i == 2 ? 0 : i - 3; }
    template <int i>
    __device__ static int pbase(const View& v) { return pair_slot(i) * v.pitch * 4; }
    template <int p>
    __device__ static int poff(const View& v) {
        if constexpr (p == 1) return (int)v.g0_offset - v.pitch * 12;
        else if constexpr (p == 3) return (int)v.g0_offset - v.pitch * 8;
        else if constexpr (p == 0) return (int)v.g0_offset - v.pitch * 4;
        else if constexpr (p < 9) return pbase<p>(v);            // low half of a pair
        else if constexpr (p == 9) return (int)v.g0_offset;
        else if constexpr (p == 10) return v.pitch * 24;         // g_1
        else if constexpr (p == 12) return v.pitch * 26;         // g_3
        else return pbase<p - 9>(v) + 2;                         // high half of a pair
    }
    // Multiplier of the 2-byte column offsets: 1 for the 16-bit planes g_1,
    // g_3, 2 for the 4-byte columns of the pair words and 32-bit planes.
    template <int p>
    static constexpr uint32_t colmul() { return (p == 10 || p == 12) ? 1 : 2; }
    __device__ static float h2f(uint16_t h) {
        if constexpr (S == ST_F16S) return (float)__builtin_bit_cast(_Float16, h);
        else return bf16_to_float(h);
    }
    __device__ static uint16_t f2h(float x) {
        if constexpr (S == ST_F16S) return __builtin_bit_cast(uint16_t, (_Float16)x);
        else return float_to_bf16(x);
    }
    // A stored element times inv = 2^-k, exact. Written as fma(h, inv, +0) so
    // that FP16 widens and scales in one mixed-precision FMA instead of a
    // convert and a multiply; the only difference from h * inv is that a -0
    // element comes out as +0.
    __device__ static float unscale(uint16_t h, float inv) {
        return __builtin_fmaf(h2f(h), inv, 0.0f);
    }
    template <int p>
    __device__ static real dec(E<p> x) {
        static_assert(p != 9, "g_0 goes through G0Code");
        if constexpr (wide(p)) return x;
        else if constexpr (p < 9) return unscale(x, 1.0f / kF);
        else return unscale(x, 1.0f / kG);
    }
    template <int p>
    __device__ static E<p> enc(real x) {
        static_assert(p != 9, "g_0 goes through G0Code");
        if constexpr (wide(p)) return x;
        else if constexpr (p < 9) return f2h(x * kF);
        else return f2h(x * kG);
    }
};
template <>
struct Fmt<ST_F16S> : Fmt16<ST_F16S> {};
template <>
struct Fmt<ST_BF16S> : Fmt16<ST_BF16S> {};

// Compressed g (tau_phi = 1): f as in FP64 / FP32; after f_0..f_8 the row block
// holds four planes with the node's g-state: phi (plane 9; in the FP32 form
// split as b + q by G0Code), Gamma mu (10) and the velocity of g^eq (11, 12).
template <>
struct Fmt<ST_F64C> : Fmt<ST_F64> {
    static constexpr bool gstate = true;
};
template <>
struct Fmt<ST_F32C> : Fmt<ST_F32> {
    static constexpr bool gstate = true;
};

// Addressing. A row block of a population buffer is reached through a buffer
// resource (base = the block, record count = its size, so the hardware
// bounds-checks every access to that row); a plane inside the block is a
// uniform scalar offset, and the column a 32-bit per-lane byte offset. Loads and
// stores are then "buffer ... offen" with no per-lane 64-bit address math.
using Rsrc = __amdgpu_buffer_rsrc_t;
constexpr int kRsrcWord3 = 0x00020000;  // raw (untyped) buffer access on gfx9-family GPUs

__device__ inline Rsrc row_rsrc(const char* buf, const View& v, int y) {
    return __builtin_amdgcn_make_buffer_rsrc((void*)(buf + (size_t)y * v.row_bytes), 0,
                                             (int)v.row_bytes, kRsrcWord3);
}

// Rows y, y-1, y+1 of the source buffer.
struct Rows {
    Rsrc r[3];
};
__device__ inline Rows rows_of(const char* buf, const View& v, int y, int ym, int yp) {
    return Rows{{row_rsrc(buf, v, y), row_rsrc(buf, v, ym), row_rsrc(buf, v, yp)}};
}

// Per-lane byte offsets: columns x, x-1, x+1 of the main element size (that of
// f_2; planes with wider columns scale them, Fmt::colmul) and column x of
// plane 9.
struct ColOff {
    uint32_t c[3];
    uint32_t c9;
};
template <int S>
__device__ inline ColOff col_offsets(uint32_t x, uint32_t xm, uint32_t xp) {
    constexpr uint32_t sz = sizeof(typename Fmt<S>::template E<2>);
    constexpr uint32_t sz9 = sizeof(typename Fmt<S>::template E<9>);
    return ColOff{{x * sz, xm * sz, xp * sz}, x * sz9};
}

// Cache-policy bits of the population loads and stores (bit 1 = nt, the
// streaming hint). Stores are nontemporal: a post-collision population is read
// again only in the next sweep, after the whole lattice has passed through the
// caches, so keeping it there only displaces lines of rows still being pulled.
#ifndef LB_LOAD_AUX
#define LB_LOAD_AUX 0
#endif
#ifndef LB_STORE_AUX
#define LB_STORE_AUX 2
#endif

template <class E>
__device__ inline E buf_ld(Rsrc r, uint32_t voff, int soff) {
    if constexpr (sizeof(E) == 8)
        return __builtin_bit_cast(
            E, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, LB_LOAD_AUX));
    else if constexpr (sizeof(E) == 4)
        return __builtin_bit_cast(
            E, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, LB_LOAD_AUX));
    else
        return __builtin_bit_cast(
            E, __builtin_amdgcn_raw_buffer_load_b16(r, voff, soff, LB_LOAD_AUX));
}

template <class E>
__device__ inline void buf_st(E x, Rsrc r, uint32_t voff, int soff) {
    if constexpr (sizeof(E) == 8)
        __builtin_amdgcn_raw_buffer_store_b64(
            __builtin_bit_cast(unsigned int __attribute__((ext_vector_type(2))), x), r, voff, soff,
            LB_STORE_AUX);
    else if constexpr (sizeof(E) == 4)
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned int, x), r, voff, soff,
                                              LB_STORE_AUX);
    else
        __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(unsigned short, x), r, voff, soff,
                                              LB_STORE_AUX);
}

// Plane p of the row behind r, at column selector c (0: x, 1: x-1, 2: x+1).
template <int S, int p>
__device__ inline typename Fmt<S>::real ldp(Rsrc r, const View& v, const ColOff& co, int c) {
    using E = typename Fmt<S>::template E<p>;
    const uint32_t voff = p == 9 ? co.c9 : co.c[c] * Fmt<S>::template colmul<p>();
    return Fmt<S>::template dec<p>(buf_ld<E>(r, voff, Fmt<S>::template poff<p>(v)));
}

template <int S, int p>
__device__ inline void stp(Rsrc r, const View& v, const ColOff& co, typename Fmt<S>::real x) {
    using E = typename Fmt<S>::template E<p>;
    buf_st<E>(Fmt<S>::template enc<p>(x), r, p == 9 ? co.c9 : co.c[0] * Fmt<S>::template colmul<p>(),
              Fmt<S>::template poff<p>(v));
}

__device__ inline int wrap(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }
// Row index v modulo n for any v: the sweep's look-ahead rows can lie more than
// one lattice height beyond a short lattice's rows (n >= 3, reach up to 3 rows
// past a strip of one row).
__device__ inline int wrap_row(int v, int n) {
    v %= n;
    return v < 0 ? v + n : v;
}

template <int N, class F>
__device__ inline void static_for(F&& f) {
    if constexpr (N > 0) {
        static_for<N - 1>(f);
        f(std::integral_constant<int, N - 1>{});
    }
}

// Read modes of the pulls (M): 0 = two buffers (the post-collision f_i of node
// r at r in plane i); 1 and 2 = the two phases of the in-place update (layout
// X: f'_i of r at r in plane OPP(i); layout P: the arriving f_i at r in plane i).
// Row selector (0: y, 1: y-1, 2: y+1) and column selector of the source of the
// population of direction i, and the plane it is read from.
template <int M, int i>
constexpr int src_row() { return M == 2 ? 0 : (EY[i] > 0 ? 1 : (EY[i] < 0 ? 2 : 0)); }
template <int M, int i>
constexpr int src_col() { return M == 2 ? 0 : (EX[i] > 0 ? 1 : (EX[i] < 0 ? 2 : 0)); }
template <int M, int i>
constexpr int src_plane() { return M == 1 ? OPP[i] : i; }
// Plane that holds, at r itself, the value pulled across a solid link i (the
// node's own post-collision value in the opposite direction).
template <int M, int i>
constexpr int bounce_plane() { return M == 1 ? i : OPP[i]; }

// Pull the nine populations of set B (0 = f, 9 = g) arriving at fluid node
// (x, y): from r - e_i, then, for links whose source is solid (bits of nb),
// the node's own post-collision value in the opposite direction (mid-link
// bounce-back). Working values (deviations for shifted f). In read mode 2 the
// arriving populations, bounce-back included, are already at r.
// For g in the shifted formats out[0] is the small part q of g_0 and *base its
// b (G0Code); otherwise *base is 0.
template <int S, int B, int M = 0>
__device__ inline void pull9(const Rows& R, const View& v, const ColOff& co, uint32_t nb,
                             typename Fmt<S>::real out[9],
                             typename Fmt<S>::real* base = nullptr) {
    using F = Fmt<S>;
    static_for<9>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        constexpr int r = src_row<M, i>();
        constexpr int c = src_col<M, i>();
        if constexpr (B == 9 && i == 0 && F::shifted) {
            const uint32_t u = buf_ld<uint32_t>(R.r[0], co.c9, F::template poff<9>(v));
            out[0] = G0Code::q(u);
            if (base) *base = G0Code::b(u);
        } else {
            out[i] = ldp<S, B + src_plane<M, i>()>(R.r[r], v, co, c);
            if (B == 9 && i == 0 && base) *base = 0;
        }
    });
    if (M != 2 && nb != 0u) {
        static_for<9>([&](auto ic) {
            constexpr int i = decltype(ic)::value;
            if constexpr (i > 0) {
                if ((nb >> (i - 1)) & 1u) out[i] = ldp<S, B + bounce_plane<M, i>()>(R.r[0], v, co, 0);
            }
        });
    }
}

// 16-bit formats: the populations arriving at fluid node (x, y) that the sweep
// takes together with phi: the paired f_i (i = 2, 4..8) into fo[i], and g into
// go (go[0] = q of g_0, base its b). f_0, f_1, f_3 are pulled separately.
// pairs_issue loads the words (the pair words, the G0Code of g_0, the 16-bit
// g_1 and g_3) and pairs_decode turns them into values, taking the bounce-back
// ones from the node itself; the sweep issues the loads one step before it
// decodes them.
template <int S>
__device__ inline void pairs_issue(const Rows& R, const View& v, const ColOff& co,
                                   uint32_t raw[9]) {
    using F = Fmt<S>;
    static_for<9>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        constexpr int r = EY[i] > 0 ? 1 : (EY[i] < 0 ? 2 : 0);
        constexpr int c = EX[i] > 0 ? 1 : (EX[i] < 0 ? 2 : 0);
        if constexpr (F::paired(i)) {
            raw[i] = buf_ld<uint32_t>(R.r[r], co.c[c] * 2, F::template pbase<i>(v));
        } else if constexpr (i == 0) {
            raw[0] = buf_ld<uint32_t>(R.r[0], co.c9, F::template poff<9>(v));
        } else {
            using E = typename F::template E<9 + i>;
            raw[i] = buf_ld<E>(R.r[r], co.c[c] * F::template colmul<9 + i>(),
                               F::template poff<9 + i>(v));
        }
    });
}

template <int S>
__device__ inline void pairs_decode(const Rows& R, const View& v, const ColOff& co, uint32_t nb,
                                    const uint32_t raw[9], float fo[9], float go[9],
                                    float& base) {
    using F = Fmt<S>;
    static_for<9>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        if constexpr (F::paired(i)) {
            fo[i] = F::unscale((uint16_t)(raw[i] & 0xFFFFu), 1.0f / F::kF);
            go[i] = F::unscale((uint16_t)(raw[i] >> 16), 1.0f / F::kG);
        } else if constexpr (i == 0) {
            go[0] = G0Code::q(raw[0]);
            base = G0Code::b(raw[0]);
        } else {
            go[i] = F::template dec<9 + i>((typename F::template E<9 + i>)raw[i]);
        }
    });
    if (nb != 0u) {
        static_for<9>([&](auto ic) {
            constexpr int i = decltype(ic)::value;
            if constexpr (i > 0) {
                if ((nb >> (i - 1)) & 1u) {
                    // the node's own post-collision values in the opposite direction
                    if constexpr (F::paired(i) && F::paired(OPP[i])) {
                        const uint32_t w =
                            buf_ld<uint32_t>(R.r[0], co.c[0] * 2, F::template pbase<OPP[i]>(v));
                        fo[i] = F::unscale((uint16_t)(w & 0xFFFFu), 1.0f / F::kF);
                        go[i] = F::unscale((uint16_t)(w >> 16), 1.0f / F::kG);
                    } else if constexpr (F::paired(i)) {
                        fo[i] = ldp<S, OPP[i]>(R.r[0], v, co, 0);
                        go[i] = ldp<S, 9 + OPP[i]>(R.r[0], v, co, 0);
                    } else {
                        go[i] = ldp<S, 9 + OPP[i]>(R.r[0], v, co, 0);
                    }
                }
            }
        });
    }
}

// Plain formats (FP64, FP32) with tau_phi = 1, two buffers: g_issue loads the
// words of the nine g pulled at (x, y) and g_finish forms phi from them with
// the arithmetic of phi9 (read mode 0). The sweep issues the loads of a ring
// row's column and of its halo column before it waits for either, and without
// waiting for the node's mask first.
template <int S>
struct GWords {
    typename Fmt<S>::template E<9> w0;
    typename Fmt<S>::template E<10> w[9];
};
template <int S>
__device__ inline void g_issue(const Rows& R, const View& v, const ColOff& co, GWords<S>& o) {
    using F = Fmt<S>;
    o.w0 = buf_ld<typename F::template E<9>>(R.r[0], co.c9, F::template poff<9>(v));
    static_for<9>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        if constexpr (i > 0) {
            using E = typename F::template E<9 + i>;
            o.w[i] = buf_ld<E>(R.r[src_row<0, i>()], co.c[src_col<0, i>()],
                               F::template poff<9 + i>(v));
        }
    });
}
template <int S>
__device__ inline typename Fmt<S>::real g_finish(const Rows& R, const View& v, const ColOff& co,
                                                 uint32_t nb, const GWords<S>& o,
                                                 typename Fmt<S>::real& small,
                                                 typename Fmt<S>::real& base) {
    using F = Fmt<S>;
    using real = typename F::real;
    real gv[9];
    if constexpr (F::shifted) {
        gv[0] = G0Code::q(o.w0);
        base = G0Code::b(o.w0);
    } else {
        gv[0] = (real)o.w0;
        base = 0;
    }
#pragma unroll
    for (int i = 1; i < 9; ++i) gv[i] = (real)o.w[i];
    if (nb != 0u) {
        static_for<9>([&](auto ic) {
            constexpr int i = decltype(ic)::value;
            if constexpr (i > 0) {
                using E = typename F::template E<9 + OPP[i]>;
                if ((nb >> (i - 1)) & 1u)
                    gv[i] = (real)buf_ld<E>(R.r[0], co.c[0], F::template poff<9 + OPP[i]>(v));
            }
        });
    }
    real sg = 0;
#pragma unroll
    for (int i = 1; i < 9; ++i) sg += gv[i];
    small = gv[0] + sg;
    return F::shifted ? base + small : small;
}

template <int S>
__device__ inline void pull_pairs(const Rows& R, const View& v, const ColOff& co, uint32_t nb,
                                  float fo[9], float go[9], float& base) {
    uint32_t raw[9];
    pairs_issue<S>(R, v, co, raw);
    pairs_decode<S>(R, v, co, nb, raw, fo, go, base);
}

// phi = sum of the nine g pulled at (x, y), for callers that need only phi.
// In the 16-bit formats the g_1..g_8 scale is applied once to their sum. In the
// shifted formats phi = base + small, small = q + g_1 + ... + g_8 (G0Code); the
// FP64 format returns small = phi, base = 0.
template <int S, int M = 0>
__device__ inline typename Fmt<S>::real phi9(const Rows& R, const View& v, const ColOff& co,
                                             uint32_t nb, typename Fmt<S>::real& small,
                                             typename Fmt<S>::real& base) {
    using F = Fmt<S>;
    using real = typename F::real;
    real gv[9];
    static_for<9>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        constexpr int r = src_row<M, i>();
        constexpr int c = src_col<M, i>();
        constexpr int pl = 9 + src_plane<M, i>();
        using E = typename F::template E<pl>;
        const E e = buf_ld<E>(R.r[r], i == 0 ? co.c9 : co.c[c], F::template poff<pl>(v));
        if constexpr (i == 0 && F::shifted) {
            gv[0] = G0Code::q(e);
            base = G0Code::b(e);
        } else if constexpr (std::is_same<E, uint16_t>::value) {
            gv[i] = Fmt16<S>::h2f(e);
        } else {
            gv[i] = (real)e;
        }
    });
    if (M != 2 && nb != 0u) {
        static_for<9>([&](auto ic) {
            constexpr int i = decltype(ic)::value;
            if constexpr (i > 0) {
                constexpr int pl = 9 + bounce_plane<M, i>();
                using E = typename F::template E<pl>;
                if ((nb >> (i - 1)) & 1u) {
                    const E e = buf_ld<E>(R.r[0], co.c[0], F::template poff<pl>(v));
                    if constexpr (std::is_same<E, uint16_t>::value) gv[i] = Fmt16<S>::h2f(e);
                    else gv[i] = (real)e;
                }
            }
        });
    }
    real s = 0;
#pragma unroll
    for (int i = 1; i < 9; ++i) s += gv[i];
    if constexpr (std::is_same<typename F::template E<10>, uint16_t>::value)
        small = gv[0] + s * (real)(1.0 / 1024.0);
    else
        small = gv[0] + s;
    if constexpr (!F::shifted) base = 0;
    return F::shifted ? base + small : small;
}

// g^eq_i of Appendix A for a node whose g-state is (phi, Gamma mu, u): the
// one expression that both the node sending g^eq_i and the node receiving it
// evaluate, so both obtain the same value bit for bit (compressed formats).
template <int i, class R>
__device__ inline R geq_dir(R ph, R gm, R ux, R uy) {
    constexpr double w = i < 5 ? 1.0 / 3.0 : 1.0 / 12.0;
    const R eu = (R)EX[i] * ux + (R)EY[i] * uy;
    const R bq = gm - (R)0.5 * ph * (ux * ux + uy * uy);
    return (R)w * (bq + (R)1.5 * ph * eu * eu) + (R)w * ph * eu;
}

template <class real>
__device__ inline real recip(real x) {
    if constexpr (std::is_same<real, float>::value) return __builtin_amdgcn_rcpf(x);
    else return (real)1 / x;
}

// Waves per SIMD the register allocator must leave room for (memory-level
// parallelism of this bandwidth-bound sweep comes from resident waves).
#ifndef LB_WAVES_F64
#define LB_WAVES_F64 2
#endif
#ifndef LB_WAVES_F32
#define LB_WAVES_F32 4
#endif
#ifndef LB_WAVES_16
#define LB_WAVES_16 LB_WAVES_F32
#endif
template <int S>
constexpr int kWaves = (S == ST_F64 || S == ST_F64C)
                           ? LB_WAVES_F64
                           : ((S == ST_F32 || S == ST_F32C) ? LB_WAVES_F32 : LB_WAVES_16);

// G1: tau_phi == 1 (the paper's choice for g), so g' = g^eq and the pulled g
// are needed only for phi; they are then not kept in registers.
// M: read mode (0: two buffers; 1, 2: the phases of the in-place update). In
// place, a workgroup forms phi only at the nodes it collides; phi at the other
// nodes of its stencil rows (the rows beyond the ends of its strip, the halo
// columns, the wrapped columns of idle lanes) comes from the band plane that
// the pre-pass of this step wrote, since their slots may already hold the
// populations of the next step.
//
// sweep_tile is one workgroup's share of a step: columns tx*BX .. tx*BX+BX-1 and
// rows y0 .. y1-1 of lattice `member`, strip index ty (odd strips walk
// downwards), read from buf[parity], written to the other buffer; tile_id is
// its partial-sum record.
template <int S, int COLL, int BX, bool DIAG, bool G1, int M>
__device__ __forceinline__ void sweep_tile(const View* __restrict__ views, int member, int tx,
                                           int ty, int ty0, int ty1, int tile_id, int parity,
                                           double* __restrict__ partials) {
    using F = Fmt<S>;
    using real = typename F::real;
    constexpr int W = BX + 4;
    __shared__ real sphi[kNR][W];
    // Compressed g: a ring of four g-state rows of the source buffer (phi word,
    // Gamma mu, u_x, u_y), with three halo columns on each side.
    using SW = typename std::conditional<S == ST_F64C, double, float>::type;
    constexpr int kGS = F::gstate ? 4 : 1, kGW = F::gstate ? BX + 6 : 1;
    __shared__ SW sst[kGS][4][kGW];

    const View v = views[member];  // uniform: lives in scalar registers
    const int nx = v.nx, ny = v.ny;
    // ?: rather than indexing buf[] by a runtime value (which would put the
    // View copy in private memory).
    const char* src = parity ? v.buf[1] : v.buf[0];
    char* dst = parity ? v.buf[0] : v.buf[1];

    const int t = threadIdx.x;
    // With lattice-node bounce-back the fluid nodes pull across every link
    // (the solid neighbour is a wall node holding the population; wall_kernel
    // fills it), so the mid-link bounce bits are dropped from the pulls.
    auto pull_mask = [&](uint32_t m) -> uint32_t {
        if constexpr ((S == ST_F64 || S == ST_F32) && M == 0) return v.bounce ? 0u : m;
        return m;
    };
    const int x0 = tx * BX;
    const int y0 = ty0;
    const int y1 = min(ty1, ny);
    const int d = (ty & 1) ? -1 : 1;  // walking direction of this strip
    const bool active = x0 + t < nx;
    // Lanes past the right edge hold wrapped columns; only the first two of
    // them (lanes nx - x0 and nx - x0 + 1) are read, by the stencil and the
    // ghost values of the last active columns, so the others skip their pulls
    // (narrow lattices on wide tiles).
    const bool used = x0 + t <= nx + 1;
    // Lanes past the right edge compute phi of the wrapped columns the
    // stencil of the last active columns needs.
    const uint32_t x = (uint32_t)((x0 + t) % nx);
    const uint32_t xm = x == 0 ? nx - 1 : x - 1;
    const uint32_t xp = x == (uint32_t)nx - 1 ? 0 : x + 1;
    // Threads 0..3 also compute phi of the halo columns x0-2, x0-1, x0+BX,
    // x0+BX+1. The stencil and ghost values of the active columns read up to
    // column nx + 1, so in a partial tile the right pair is skipped where it
    // lies beyond that (the wrapped lanes hold those columns). (Spreading
    // these over the wavefronts measured slower.)
    const bool halo = t < 2 || (t < 4 && x0 + BX + t - 2 <= nx + 1);
    const int hcol = t < 2 ? t : BX + t;
    const uint32_t hx = (uint32_t)(((x0 - 2 + hcol) % nx + nx) % nx);
    const uint32_t hxm = hx == 0 ? nx - 1 : hx - 1;
    const uint32_t hxp = hx == (uint32_t)nx - 1 ? 0 : hx + 1;

    const real rA = (real)v.A, rB = (real)v.B, rK = (real)v.kappa, rG = (real)v.Gamma;
    const real ta = (real)v.tau_alpha, tb = (real)v.tau_beta, itp = (real)v.inv_tau_phi;
    const real rApB = (real)(v.A + v.B);
    const real rho_ref = (real)v.rho_ref;
    const GLOBAL uint8_t* nbr = (const GLOBAL uint8_t*)v.nbr;
    const GLOBAL uint8_t* grec = (const GLOBAL uint8_t*)v.grec;
    // Wall gradients are FP64 for the FP64 format and FP32 otherwise.
    using DW = typename std::conditional<S == ST_F64 || S == ST_F64C, double, float>::type;
    const GLOBAL DW* dphi = (const GLOBAL DW*)v.dphi;

    const ColOff co = col_offsets<S>(x, xm, xp);
    const ColOff hco = col_offsets<S>(hx, hxm, hxp);

    // phi at the columns of `c` of the row behind R; the nine pulled g are
    // returned in g unless G1.
    // (small, base): see phi9. In the 16-bit formats the paired f_i arrive
    // with the g and are returned in fp.
    auto phi_of = [&](const Rows& R, uint32_t nb, const ColOff& c, real g[9], real fp[9],
                      real& small, real& base) -> real {
        small = 0;
        base = 0;
        if (nb == 0xFFu) return (real)0;
        if constexpr (F::packed) {
            pull_pairs<S>(R, v, c, nb, fp, g, base);
#pragma unroll
            for (int i = 0; i < 9; ++i) small += g[i];
            return base + small;
        } else if constexpr (G1) {
            return phi9<S, M>(R, v, c, pull_mask(nb), small, base);
        } else {
            pull9<S, 9, M>(R, v, c, pull_mask(nb), g, &base);
#pragma unroll
            for (int i = 0; i < 9; ++i) small += g[i];
            return base + small;
        }
    };
    // Compressed g: load g-state row yy into the ring (this thread's column;
    // threads 0..5 also the halo columns x0-3..x0-1, x0+BX..x0+BX+2).
    // threads 0..5 load the six halo columns of the g-state
    const bool shalo = t < 6;
    const int scol = t < 3 ? t : BX + t;
    const uint32_t sx = (uint32_t)(((x0 - 3 + scol) % nx + nx) % nx);
    // The state columns the used lanes read.
    const bool sused = x0 + t <= nx + 2;
    // state_issue loads row yy into registers (stM, and stH for the halo
    // lanes); state_commit writes the registers of the row loaded last into
    // the ring. The sweep commits a row one step after issuing it, so its
    // loads are in flight during a row of arithmetic.
    SW stM[F::gstate ? 4 : 1], stH[F::gstate ? 4 : 1];
    auto state_issue = [&](int yy) __attribute__((always_inline)) {
        if constexpr (F::gstate) {
            const Rsrc rr = row_rsrc(src, v, wrap_row(yy, ny));
            auto ld = [&](uint32_t xx, SW* o) {
                if constexpr (S == ST_F32C)
                    o[0] = __builtin_bit_cast(
                        float, buf_ld<uint32_t>(rr, xx * 4, F::template poff<9>(v)));
                else
                    o[0] = buf_ld<SW>(rr, xx * sizeof(SW), F::template poff<9>(v));
                o[1] = buf_ld<SW>(rr, xx * sizeof(SW), F::template poff<10>(v));
                o[2] = buf_ld<SW>(rr, xx * sizeof(SW), F::template poff<11>(v));
                o[3] = buf_ld<SW>(rr, xx * sizeof(SW), F::template poff<12>(v));
            };
            if (sused) ld(x, stM);
            if (shalo) ld(sx, stH);
        }
    };
    auto state_commit = [&](int yy) __attribute__((always_inline)) {
        if constexpr (F::gstate) {
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                if (sused) sst[yy & 3][k][t + 3] = stM[k];
                if (shalo) sst[yy & 3][k][scol] = stH[k];
            }
        }
    };
    auto load_state_row = [&](int yy) __attribute__((always_inline)) {
        state_issue(yy);
        state_commit(yy);
    };
    // g-state at ring slot sl, column col: phi = b + q and the g^eq inputs.
    auto gstate_at = [&](int sl, int col, real& ph, real& gm, real& gu, real& gv, real& q,
                         real& b) __attribute__((always_inline)) {
        if constexpr (S == ST_F32C) {
            const uint32_t u = __builtin_bit_cast(uint32_t, (float)sst[sl][0][col]);
            q = G0Code::q(u);
            b = G0Code::b(u);
            ph = b + q;
        } else {
            q = (real)sst[sl][0][col];
            b = 0;
            ph = q;
        }
        gm = (real)sst[sl][1][col];
        gu = (real)sst[sl][2][col];
        gv = (real)sst[sl][3][col];
    };
    // phi of S_{n+1} at row yy, ring column c: Eq. (stream2) with g' = g^eq
    // (tau_phi = 1) in flux form, phi + sum of g^eq_i arriving (from r - e_i, or
    // bounced back at r) - sum of g^eq_i leaving; each g^eq_i is evaluated by
    // geq_dir from the same stored state on both sides, so sum phi is kept.
    auto phi_gstate = [&](int yy, int c, uint32_t nb, real& small,
                          real& base) __attribute__((always_inline)) -> real {
        small = 0;
        base = 0;
        if (nb == 0xFFu) return (real)0;
        real ph0, gm0, gu0, gv0, q0, b0;
        gstate_at(yy & 3, c, ph0, gm0, gu0, gv0, q0, b0);
        real out = 0, in = 0;
        static_for<9>([&](auto ic) {
            constexpr int i = decltype(ic)::value;
            if constexpr (i > 0) {
                out += geq_dir<i>(ph0, gm0, gu0, gv0);
                if ((nb >> (i - 1)) & 1u) {
                    in += geq_dir<OPP[i]>(ph0, gm0, gu0, gv0);
                } else {
                    real ph1, gm1, gu1, gv1, q1, b1;
                    gstate_at((yy - EY[i]) & 3, c - EX[i], ph1, gm1, gu1, gv1, q1, b1);
                    in += geq_dir<i>(ph1, gm1, gu1, gv1);
                }
            }
        });
        small = q0 + (in - out);
        base = b0;
        return base + small;
    };
    // FP64 / FP32 with tau_phi = 1, two buffers: ring row yy in two halves.
    // g_row_issue loads the masks and the g words of this column and of the
    // halo column, all before anything waits for them; g_row_finish forms phi
    // from them into the ring.
    auto g_row_issue = [&](int yy, GWords<S>& wM, GWords<S>& wH, uint32_t& nbm,
                           uint32_t& nbh) __attribute__((always_inline)) {
        const int y = wrap_row(yy, ny);
        const GLOBAL uint8_t* nrow = nbr + (size_t)y * v.pitch;
        const Rows R = rows_of(src, v, y, wrap(y - 1, ny), wrap(y + 1, ny));
        nbm = used ? nrow[x] : 0xFFu;
        nbh = halo ? nrow[hx] : 0xFFu;
        if (used) g_issue<S>(R, v, co, wM);
        if (halo) g_issue<S>(R, v, hco, wH);
    };
    auto g_row_finish = [&](int yy, const GWords<S>& wM, const GWords<S>& wH, uint32_t nbm,
                            uint32_t nbh, real& small, real& base) __attribute__((always_inline)) {
        const int y = wrap_row(yy, ny);
        const Rows R = rows_of(src, v, y, wrap(y - 1, ny), wrap(y + 1, ny));
        small = 0;
        base = 0;
        real ph = 0;
        if (nbm != 0xFFu) ph = g_finish<S>(R, v, co, pull_mask(nbm), wM, small, base);
        sphi[yy & (kNR - 1)][t + 2] = ph;
        if (halo) {
            real hs = 0, hb = 0, hp = 0;
            if (nbh != 0xFFu) hp = g_finish<S>(R, v, hco, pull_mask(nbh), wH, hs, hb);
            sphi[yy & (kNR - 1)][hcol] = hp;
        }
    };
    // Fill ring row yy: this thread's column and the halo columns.
    auto fill_row = [&](int yy, real g[9], real fp[9], uint32_t& nb, real& small,
                        real& base) __attribute__((always_inline)) {
        if constexpr (F::gstate) {
            // the node masks first (their wait then leaves the state loads in
            // flight), the g-state two rows further on into the ring, the
            // loads of the row after it, then phi of row yy from the state
            // rows yy - 1, yy, yy + 1 committed before
            const GLOBAL uint8_t* nrow = nbr + (size_t)wrap_row(yy, ny) * v.pitch;
            nb = nrow[x];
            const uint32_t hnb = halo ? nrow[hx] : 0xFFu;
            state_commit(yy + 2 * d);
            state_issue(yy + 3 * d);
            sphi[yy & (kNR - 1)][t + 2] = phi_gstate(yy, t + 3, nb, small, base);
            if (halo) {
                real hs, hb;
                sphi[yy & (kNR - 1)][hcol] = phi_gstate(yy, hcol + 1, hnb, hs, hb);
            }
            return;
        }
        const int y = wrap_row(yy, ny);
        const GLOBAL uint8_t* nrow = nbr + (size_t)y * v.pitch;
        nb = nrow[x];
        if constexpr (M != 0) {
            const GLOBAL real* brow = (const GLOBAL real*)v.band + (size_t)y * v.pitch;
            if (active && yy >= y0 && yy < y1) {
                const Rows R = rows_of(src, v, y, wrap(y - 1, ny), wrap(y + 1, ny));
                sphi[yy & (kNR - 1)][t + 2] = phi_of(R, nb, co, g, fp, small, base);
            } else {
                small = 0;
                base = 0;
                sphi[yy & (kNR - 1)][t + 2] = brow[x];
            }
            if (halo) sphi[yy & (kNR - 1)][hcol] = brow[hx];
            return;
        }
        if constexpr (!F::packed && G1) {
            GWords<S> wM, wH;
            uint32_t hnb;
            g_row_issue(yy, wM, wH, nb, hnb);
            g_row_finish(yy, wM, wH, nb, hnb, small, base);
            return;
        }
        const Rows R = rows_of(src, v, y, wrap(y - 1, ny), wrap(y + 1, ny));
        if (!used) nb = 0xFFu;
        sphi[yy & (kNR - 1)][t + 2] = phi_of(R, nb, co, g, fp, small, base);
        if (halo) {
            real hg[9], hf[9], hs, hb;
            sphi[yy & (kNR - 1)][hcol] = phi_of(R, nrow[hx], hco, hg, hf, hs, hb);
        }
    };

    // 16-bit formats: the loads of ring row y + 3d and of f_0, f_1, f_3 of row
    // y + d are issued while row y is collided and consumed in the next step,
    // so each row's memory latency overlaps a row of arithmetic. The words are
    // loaded whether or not the node is solid (every address is inside its
    // row): a load that waited for the node's mask would wait for every load
    // in flight, the previous row's stores included.
    constexpr bool kPF = F::packed;
    uint32_t rawM[kPF ? 9 : 1], rawH[kPF ? 9 : 1];  // words of this column, of the halo column
    uint32_t rawNbM = 0xFFu, rawNbH = 0xFFu;
    real pf0 = 0, pf1 = 0, pf3 = 0;
    // The words of ring row yy into (wm, wh, nbm, nbh): this column's, the
    // halo column's, and their masks.
    auto raw_issue_to = [&](int yy, uint32_t (&wm)[kPF ? 9 : 1], uint32_t (&wh)[kPF ? 9 : 1],
                            uint32_t& nbm, uint32_t& nbh) __attribute__((always_inline)) {
        if constexpr (kPF) {
            const int y = wrap_row(yy, ny);
            const GLOBAL uint8_t* nrow = nbr + (size_t)y * v.pitch;
            const Rows R = rows_of(src, v, y, wrap(y - 1, ny), wrap(y + 1, ny));
            nbm = used ? nrow[x] : 0xFFu;
            if (used) pairs_issue<S>(R, v, co, wm);
            if (halo) {
                nbh = nrow[hx];
                pairs_issue<S>(R, v, hco, wh);
            }
        }
    };
    // phi of ring row yy from words raw_issue_to loaded (as fill_row forms it)
    auto raw_finish_from = [&](int yy, const uint32_t (&wm)[kPF ? 9 : 1],
                               const uint32_t (&wh)[kPF ? 9 : 1], uint32_t nbm, uint32_t nbh,
                               real g[9], real fp[9], uint32_t& nb, real& small,
                               real& base) __attribute__((always_inline)) {
        if constexpr (kPF) {
            const int y = wrap_row(yy, ny);
            const Rows R = rows_of(src, v, y, wrap(y - 1, ny), wrap(y + 1, ny));
            nb = nbm;
            small = 0;
            base = 0;
            real ph = 0;
            if (nb != 0xFFu) {
                pairs_decode<S>(R, v, co, nb, wm, fp, g, base);
#pragma unroll
                for (int i = 0; i < 9; ++i) small += g[i];
                ph = base + small;
            }
            sphi[yy & (kNR - 1)][t + 2] = ph;
            if (halo) {
                real hg[9], hf[9], hs = 0, hb = 0, hp = 0;
                if (nbh != 0xFFu) {
                    pairs_decode<S>(R, v, hco, nbh, wh, hf, hg, hb);
#pragma unroll
                    for (int i = 0; i < 9; ++i) hs += hg[i];
                    hp = hb + hs;
                }
                sphi[yy & (kNR - 1)][hcol] = hp;
            }
        }
    };
    auto raw_issue = [&](int yy) __attribute__((always_inline)) {
        raw_issue_to(yy, rawM, rawH, rawNbM, rawNbH);
    };
    auto raw_finish = [&](int yy, real g[9], real fp[9], uint32_t& nb, real& small,
                          real& base) __attribute__((always_inline)) {
        raw_finish_from(yy, rawM, rawH, rawNbM, rawNbH, g, fp, nb, small, base);
    };
    // f_0, f_1, f_3 of row yy (pull sources as in the sweep; nbr_ its mask)
    auto f_issue = [&](int yy, uint32_t nbr_) __attribute__((always_inline)) {
        if constexpr (kPF) {
            if (active && nbr_ != 0xFFu) {
                const int y = wrap_row(yy, ny);
                const Rows R = rows_of(src, v, y, wrap(y - 1, ny), wrap(y + 1, ny));
                pf0 = ldp<S, 0>(R.r[0], v, co, 0);
                pf1 = (nbr_ & 1u) ? ldp<S, 2>(R.r[0], v, co, 0) : ldp<S, 1>(R.r[0], v, co, 1);
                pf3 = (nbr_ & 4u) ? ldp<S, 4>(R.r[0], v, co, 0) : ldp<S, 3>(R.r[1], v, co, 0);
            }
        }
    };

    double d_drho = 0.0, d_phi = 0.0, d_ke = 0.0, d_umax = 0.0, d_n = 0.0;

    // One row: fill the ring two rows ahead in the walking direction d
    // (gnew), then collide row y (gc). The f pulls of row y are issued before
    // the look-ahead g pulls are consumed, so both sets of loads are in flight
    // together and each row waits for memory once.
    auto step = [&](int y, real gc[9], real fc[9], uint32_t nbc, real phs, real phb,
                    real gnew[9], real fnew[9], uint32_t& nbnew, real& snew, real& bnew,
                    uint32_t nbnext) __attribute__((always_inline)) {
        const bool work = active && nbc != 0xFFu;
        const uint32_t nb = nbc;
        const Rows R = rows_of(src, v, y, wrap(y - 1, ny), wrap(y + 1, ny));
        real f[9];
        if constexpr (F::packed) {
            // f_2, f_4..f_8 came with the g of this row, f_0, f_1, f_3 were
            // loaded in the previous step. Then ring row y + 2d from the words
            // loaded in the previous step, and the loads for the next step.
            if (work) {
#pragma unroll
                for (int i = 0; i < 9; ++i) f[i] = fc[i];
                f[0] = pf0;
                f[1] = pf1;
                f[3] = pf3;
            }
            raw_finish(y + 2 * d, gnew, fnew, nbnew, snew, bnew);
            f_issue(y + d, nbnext);
            raw_issue(y + 3 * d);
        } else {
            if (work) pull9<S, 0, M>(R, v, co, pull_mask(nb), f);
            fill_row(y + 2 * d, gnew, fnew, nbnew, snew, bnew);
        }
        __syncthreads();
        if (!work) return;

        const int c = t + 2;
        const real ph = sphi[y & (kNR - 1)][c];
        // phi at the eight neighbours k = 1..8 (ghost values at solid ones).
        real pn[9];
#pragma unroll
        for (int k = 1; k < 9; ++k) pn[k] = sphi[(y + EY[k]) & (kNR - 1)][c + EX[k]];
        if (nb != 0u) {
#pragma unroll
            for (int k = 1; k < 9; ++k) {
                if ((nb >> (OPP[k] - 1)) & 1u) {
                    // Solid neighbour s = r + e_k: mean of phi over its fluid axis
                    // neighbours (else diagonal ones) minus the wall gradient (times
                    // sqrt 2 across a diagonal).
                    const int sy = wrap(y + EY[k], ny);
                    const uint32_t sxw = EX[k] == 0 ? x : (EX[k] > 0 ? xp : xm);
                    const size_t s = (size_t)sy * v.pitch + sxw;
                    const uint32_t rec = grec[s];
                    const real dw = (real)dphi[s];
                    const uint32_t axis = rec & 0xFu;
                    const uint32_t bits = axis ? axis : (rec >> 4);
                    real sum = 0;
                    int cnt = 0;
                    static_for<4>([&](auto mc) {
                        // fluid neighbour s + e_m, m = mm + 1 (axis) or mm + 5 (diagonal)
                        constexpr int mm = decltype(mc)::value;
                        constexpr int exa = EX[mm + 1], eya = EY[mm + 1];
                        constexpr int exd = EX[mm + 5], eyd = EY[mm + 5];
                        if ((bits >> mm) & 1u) {
                            const int ex = axis ? exa : exd;
                            const int ey = axis ? eya : eyd;
                            sum += sphi[(y + EY[k] + ey) & (kNR - 1)][c + EX[k] + ex];
                            ++cnt;
                        }
                    });
                    // Formed without a branch on cnt, so that the loads of rec and
                    // dw are consumed on every path through this node's code.
                    const real scale = axis ? (real)1 : (real)1.4142135623730951;
                    const real gv = sum / (real)(cnt > 0 ? cnt : 1) - scale * dw;
                    pn[k] = cnt > 0 ? gv : (real)0;
                }
            }
        }
        // Eq. (best): E = 1, W = 2, N = 3, S = 4, NE = 5, SW = 6, NW = 7, SE = 8.
        const real gx =
            ((real)4 * (pn[1] - pn[2]) + (pn[5] - pn[7]) + (pn[8] - pn[6])) * (real)(1.0 / 12.0);
        const real gy =
            ((real)4 * (pn[3] - pn[4]) + (pn[5] - pn[8]) + (pn[7] - pn[6])) * (real)(1.0 / 12.0);
        // Laplacian from differences to the centre (2 sum w_i (phi_i - phi)):
        // summing the phi ~ +-1 values first would cancel away FP32 digits.
        const real lap = ((real)4 * (((pn[1] - ph) + (pn[2] - ph)) + ((pn[3] - ph) + (pn[4] - ph))) +
                          (((pn[5] - ph) + (pn[6] - ph)) + ((pn[7] - ph) + (pn[8] - ph)))) *
                         (real)(1.0 / 6.0);

        // Moments, Eq. (moments): sums of the working values (deviations in the
        // shifted formats, whose rest state has zero momentum and mass rho_ref).
        const real srho = ((f[0] + f[1]) + (f[2] + f[3])) + ((f[4] + f[5]) + (f[6] + f[7])) + f[8];
        const real jx = (f[1] - f[2]) + (f[5] - f[6]) + (f[8] - f[7]);
        const real jy = (f[3] - f[4]) + (f[5] - f[6]) + (f[7] - f[8]);
        const real rho = F::shifted ? rho_ref + srho : srho;
        const real inv_rho = recip(rho);
        const real ux = jx * inv_rho, uy = jy * inv_rho;

        if constexpr (DIAG) {
            const double u2 = (double)ux * ux + (double)uy * uy;
            d_drho += F::shifted ? (double)srho : (double)srho - (double)v.rho_ref;
            d_phi += F::shifted ? (double)phb + (double)phs : (double)ph;
            d_ke += 0.5 * (double)rho * u2;
            const double um = sqrt(u2);
            d_umax = (um > d_umax || um != um) ? um : d_umax;
            d_n += 1.0;
        }

        // Eqs. (chempot), (p0), (tau). In the shifted formats p0 is taken
        // relative to its rest value and mu uses phi^2 - 1 = (phi - 1)(phi + 1).
        real mu, basef;
        if constexpr (F::shifted) {
            const real q = (ph - (real)1) * (ph + (real)1);
            mu = ph * (rB * q + rApB) - rK * lap;
            const real dp0 = srho * (real)(1.0 / 3.0) +
                             q * (rA * (real)0.5 + rB * (real)0.75 * (ph * ph + (real)1));
            basef = dp0 - rK * ph * lap;
        } else {
            mu = ph * (rA + rB * ph * ph) - rK * lap;
            const real p0 = rho * (real)(1.0 / 3.0) +
                            ph * ph * (rA * (real)0.5 + rB * (real)0.75 * ph * ph);
            basef = p0 - rK * ph * lap;
        }
        real tau;
        if (v.tau_lut > 1) {
            // Sec. VI table: entry k = nearest to the Eq. (tau) value, i.e. to
            // position (phi + 1) / 2 (n - 1) along the table, lower on a tie.
            const real tn = (real)(v.tau_lut - 1);
            real pos = (ph + (real)1) * (real)0.5 * tn;
            pos = pos < (real)0 ? (real)0 : (pos > tn ? tn : pos);
            tau = tb + ceil(pos - (real)0.5) * (real)v.tau_step;
        } else {
            const real pt =
                !v.tau_clamp ? ph : (ph > (real)1 ? (real)1 : (ph < (real)-1 ? (real)-1 : ph));
            tau = tb + (real)0.5 * (pt + (real)1) * (ta - tb);
        }
        const real omega = recip(tau);

        // Step 2: u = 0 at boundary nodes in the equilibria (flags).
        const bool bnd = nb != 0u;
        const bool zf = bnd && v.zero_u_feq;
        const bool zg = bnd && v.zero_u_geq;
        const real ufx = zf ? (real)0 : ux, ufy = zf ? (real)0 : uy;
        const real ugx = zg ? (real)0 : ux, ugy = zg ? (real)0 : uy;

        // Appendix A, Eq. (equilibrium), evaluated for the pairs (e_i, -e_i):
        // f^eq = even + odd and f^eq(-e) = even - odd, with the even part
        // w [base + 3/2 rho ((e.u)^2 - |u|^2/3)] + gradient terms and the odd part
        // w rho e.u; f^eq_0 from Eq. (feq0). Shifted formats: f^eq - r.
        const real gxx = rK * gx * gx, gyy = rK * gy * gy, gxy = rK * gx * gy;
        const real t3 = (real)(1.0 / 3.0), t12 = (real)(1.0 / 12.0);
        real feq[9], geq[9];
        real ev_x, ev_y, ev_p, ev_m;  // even parts of the pairs (1,2), (3,4), (5,6), (7,8)
        {
            const real usf = ufx * ufx + ufy * ufy;
            const real bq = basef - (real)0.5 * rho * usf;  // base + 3/2 rho (0 - |u|^2/3)
            const real r15 = (real)1.5 * rho;
            const real upm = ufx + ufy, umm = ufy - ufx;
            const real gd = (real)(1.0 / 24.0) * (gxx + gyy);
            ev_x = t3 * (bq + r15 * ufx * ufx) + (t3 * gxx - (real)(1.0 / 6.0) * gyy);
            ev_y = t3 * (bq + r15 * ufy * ufy) + (t3 * gyy - (real)(1.0 / 6.0) * gxx);
            ev_p = t12 * (bq + r15 * upm * upm) - gd + (real)0.25 * gxy;
            ev_m = t12 * (bq + r15 * umm * umm) - gd - (real)0.25 * gxy;
            real ox = t3 * rho * ufx, oy = t3 * rho * ufy;
            real op = t12 * rho * upm, om = t12 * rho * umm;
            if constexpr (F::shifted) {
                // The odd parts carry the momentum of f^eq, 2 (ox + op - om) and
                // 2 (oy + op + om): exactly rho u* (j, or 0 under Step 2), but in
                // FP32 rho (j / rho) and the weight sum 2/3 + 4/12 round with a
                // bias of one sign, and momentum, which the collision never
                // relaxes, would compound it from step to step. Moving the odd
                // pattern e_i (it carries momentum and no other moment) makes the
                // momentum of f^eq its target up to unbiased rounding.
                const real tx = zf ? (real)0 : jx, ty = zf ? (real)0 : jy;
                const real cx = (tx - (real)2 * ((ox + op) - om)) * (real)(1.0 / 6.0);
                const real cy = (ty - (real)2 * ((oy + op) + om)) * (real)(1.0 / 6.0);
                ox += cx;
                oy += cy;
                op += cx + cy;
                om += cy - cx;
            }
            feq[1] = ev_x + ox; feq[2] = ev_x - ox;
            feq[3] = ev_y + oy; feq[4] = ev_y - oy;
            feq[5] = ev_p + op; feq[6] = ev_p - op;
            feq[7] = ev_m + om; feq[8] = ev_m - om;
            // rho - sum (absolute) or (rho - rho_ref) - sum (shifted)
            feq[0] = srho - (real)2 * ((ev_x + ev_y) + (ev_p + ev_m));
        }
        {
            const real usg = ugx * ugx + ugy * ugy;
            const real bq = rG * mu - (real)0.5 * ph * usg;
            const real p15 = (real)1.5 * ph;
            const real upm = ugx + ugy, umm = ugy - ugx;
            const real ex_ = t3 * (bq + p15 * ugx * ugx), ey_ = t3 * (bq + p15 * ugy * ugy);
            const real ep_ = t12 * (bq + p15 * upm * upm), em_ = t12 * (bq + p15 * umm * umm);
            const real ox = t3 * ph * ugx, oy = t3 * ph * ugy;
            const real op = t12 * ph * upm, om = t12 * ph * umm;
            geq[1] = ex_ + ox; geq[2] = ex_ - ox;
            geq[3] = ey_ + oy; geq[4] = ey_ - oy;
            geq[5] = ep_ + op; geq[6] = ep_ - op;
            geq[7] = em_ + om; geq[8] = em_ - om;
            geq[0] = ph - (real)2 * ((ex_ + ey_) + (ep_ + em_));
        }

        // Collision.
        real fo[9];
        if constexpr (COLL == CO_BGK) {
#pragma unroll
            for (int i = 0; i < 9; ++i) fo[i] = f[i] - omega * (f[i] - feq[i]);
        } else {
            // Eq. (mrtlb) with S = diag(0,1,1,0,1,0,1,w,w) written in moment space:
            // f' = f^eq + (projection of f - f^eq on the conserved modes 0, 3, 5)
            //      + (1 - w)(projection on the stress modes 7, 8),
            // from the orthogonality of the rows of M (norms 9,36,36,6,12,6,12,4,4).
            // Stress moments of f - f^eq: rows 7 (e_x^2 - e_y^2) and 8 (e_x e_y).
            const real cw = (real)0.25 * ((real)1 - omega);
            const real m7 = (((f[1] + f[2]) - (f[3] + f[4])) - (real)2 * (ev_x - ev_y)) * cw;
            const real m8 = (((f[5] + f[6]) - (f[7] + f[8])) - (real)2 * (ev_p - ev_m)) * cw;
            // j - j^eq is zero unless Step 2 removed u from f^eq (in the shifted
            // formats f^eq was adjusted above so that this holds as formed).
            const real qx = zf ? jx * (real)(1.0 / 6.0) : (real)0;
            const real qy = zf ? jy * (real)(1.0 / 6.0) : (real)0;
            fo[0] = feq[0];
            fo[1] = feq[1] + m7 + qx;
            fo[2] = feq[2] + m7 - qx;
            fo[3] = feq[3] - m7 + qy;
            fo[4] = feq[4] - m7 - qy;
            fo[5] = feq[5] + m8 + qx + qy;
            fo[6] = feq[6] + m8 - qx - qy;
            fo[7] = feq[7] - m8 - qx + qy;
            fo[8] = feq[8] - m8 + qx - qy;
        }
        const Rsrc out = row_rsrc(dst, v, y);
        // Store the encoded post-collision value e of direction i of set B
        // (0 = f, 9 = g): at r in plane B + i (two buffers); in place, phase 0
        // sends it to r + e_i in plane B + i, or keeps it at r in plane
        // B + OPP(i) when r + e_i is solid, and phase 1 keeps it at r in plane
        // B + OPP(i) (the layouts of the next read).
        auto put = [&](auto bc, auto ic, auto e) __attribute__((always_inline)) {
            constexpr int B = decltype(bc)::value, i = decltype(ic)::value;
            using E = decltype(e);
            constexpr int pi = B + i, po = B + OPP[i];
            const uint32_t own = pi == 9 ? co.c9 : co.c[0] * F::template colmul<pi>();
            if constexpr (M == 0) {
                buf_st<E>(e, out, own, F::template poff<pi>(v));
            } else if constexpr (M == 2 || i == 0) {
                buf_st<E>(e, out, own, F::template poff<po>(v));
            } else {
                if ((nb >> (OPP[i] - 1)) & 1u) {
                    buf_st<E>(e, out, own, F::template poff<po>(v));
                } else {
                    constexpr int rr = EY[i] > 0 ? 2 : (EY[i] < 0 ? 1 : 0);
                    constexpr int cc = EX[i] > 0 ? 2 : (EX[i] < 0 ? 1 : 0);
                    const int yd = rr == 0 ? y : wrap(y + EY[i], ny);
                    buf_st<E>(e, row_rsrc(dst, v, yd), co.c[cc] * F::template colmul<pi>(),
                              F::template poff<pi>(v));
                }
            }
        };
        using IC0 = std::integral_constant<int, 0>;
        using IC9 = std::integral_constant<int, 9>;
        if constexpr (F::packed) {
            // Mass- and momentum-preserving encoding: f_2, f_4..f_8 are rounded
            // to 16 bits first; the 32-bit f_1 and f_3 are then set so that the
            // stored set carries the post-collision momentum, and the 32-bit f_0
            // so that it carries the node's mass (collision conserves it). The
            // exact f'_1, f'_3, f'_0 satisfy the same relations before rounding.
            // g_1..g_8 (Eq. (gevo); g^eq when tau_phi = 1) are rounded, and g_0
            // is phi minus their stored sum (G0Code).
            const real tx = (fo[1] - fo[2]) + (fo[5] - fo[6]) + (fo[8] - fo[7]);
            const real ty = (fo[3] - fo[4]) + (fo[5] - fo[6]) + (fo[7] - fo[8]);
            float r[9];
            uint32_t hf[9], hg[9];
            real sg = 0;
            static_for<9>([&](auto ic) {
                constexpr int i = decltype(ic)::value;
                if constexpr (F::paired(i)) {
                    hf[i] = F::f2h(fo[i] * F::kF);
                    r[i] = F::unscale((uint16_t)hf[i], 1.0f / F::kF);
                }
                if constexpr (i > 0) {
                    const real gi = G1 ? geq[i] : gc[i] - itp * (gc[i] - geq[i]);
                    hg[i] = F::f2h(gi * F::kG);
                    sg += F::h2f((uint16_t)hg[i]);
                }
            });
            static_for<9>([&](auto ic) {
                constexpr int i = decltype(ic)::value;
                if constexpr (F::paired(i))
                    buf_st<uint32_t>(hf[i] | (hg[i] << 16), out, co.c[0] * 2,
                                     F::template pbase<i>(v));
            });
            buf_st<uint16_t>((uint16_t)hg[1], out, co.c[0], F::template poff<10>(v));
            buf_st<uint16_t>((uint16_t)hg[3], out, co.c[0], F::template poff<12>(v));
            const float f1 = tx - (((r[5] - r[6]) + (r[8] - r[7])) - r[2]);
            const float f3 = ty - (((r[5] - r[6]) + (r[7] - r[8])) - r[4]);
            buf_st<float>(f1, out, co.c9, F::template poff<1>(v));
            buf_st<float>(f3, out, co.c9, F::template poff<3>(v));
            const float f0 = srho - (((f1 + r[2]) + (f3 + r[4])) + ((r[5] + r[6]) + (r[7] + r[8])));
            buf_st<float>(f0, out, co.c9, F::template poff<0>(v));
            real q = phs - sg * (1.0f / F::kG), b = phb;
            G0Code::rebase(q, b);
            buf_st<uint32_t>(G0Code::enc(q, b), out, co.c9, F::template poff<9>(v));
        } else {
            static_for<9>([&](auto ic) {
                constexpr int i = decltype(ic)::value;
                put(IC0{}, ic, F::template enc<i>(fo[i]));
            });
        }
        if constexpr (F::gstate) {
            // g-state of the node for the next step: phi of S_{n+1} (this
            // row's phi), Gamma mu and the velocity of g^eq (Step 2 flag).
            if constexpr (S == ST_F32C) {
                real q = phs, b = phb;
                G0Code::rebase(q, b);
                buf_st<uint32_t>(G0Code::enc(q, b), out, co.c9, F::template poff<9>(v));
            } else {
                stp<S, 9>(out, v, co, phs);
            }
            stp<S, 10>(out, v, co, rG * mu);
            stp<S, 11>(out, v, co, ugx);
            stp<S, 12>(out, v, co, ugy);
        } else if constexpr (F::packed) {
        } else if constexpr (F::shifted) {
            // Eq. (gevo) for g_1..g_8 (with tau_phi = 1 exactly g^eq); g_0 is
            // phi minus their stored sum, formed from the small parts (BGK for g
            // conserves phi, so this is the exact g'_0).
            real sg = 0;
            static_for<8>([&](auto ic) {
                constexpr int i = decltype(ic)::value + 1;
                using E = typename F::template E<9 + i>;
                const real gi = G1 ? geq[i] : gc[i] - itp * (gc[i] - geq[i]);
                const E e = F::template enc<9 + i>(gi);
                if constexpr (std::is_same<E, uint16_t>::value) sg += Fmt16<S>::h2f(e);
                else sg += e;
                put(IC9{}, std::integral_constant<int, i>{}, e);
            });
            if constexpr (std::is_same<typename F::template E<10>, uint16_t>::value)
                sg *= (real)(1.0 / 1024.0);
            real q = phs - sg, b = phb;
            G0Code::rebase(q, b);
            buf_st<uint32_t>(G0Code::enc(q, b), out, co.c9, F::template poff<9>(v));
        } else {
            static_for<9>([&](auto ic) {
                constexpr int i = decltype(ic)::value;
                // Eq. (gevo); with tau_phi = 1 exactly g^eq.
                put(IC9{}, ic, F::template enc<9 + i>(G1 ? geq[i] : gc[i] - itp * (gc[i] - geq[i])));
            });
        }
    };

    real gA[9], gB[9], gC[9];
    real fA[9], fB[9], fC[9];     // paired f of the 16-bit formats
    uint32_t nbA, nbB, nbC;
    real sA, sB, sC, bA, bB, bC;  // phi = b + s of this column (see phi9)
    // Odd strips walk downwards, so the two strips on either side of a strip
    // boundary reach the rows they share (the halo of the phi stencil) at the
    // same time and the second read hits in L2: vertical neighbours are
    // gridDim.x workgroups apart and share an XCD when gridDim.x % 8 == 0.
    const int nrow = y1 - y0;
    const int ys = (d > 0) ? y0 : y1 - 1;
    if constexpr (F::gstate) {
        // the state rows the first phi row needs; each later fill reads rows
        // written by other threads in the fill before it
        load_state_row(ys - 3 * d);
        load_state_row(ys - 2 * d);
        load_state_row(ys - d);
        state_issue(ys);
        __syncthreads();
    }
    if constexpr (kPF) {
        // the first four ring rows two at a time: both rows' loads are in
        // flight before either is decoded (the second set of words lives only
        // here); f of the first collided row is issued with the fourth row
        real gt[9], ft[9], st, bt;
        uint32_t nbt, w2m[9], w2h[9], n2m = 0xFFu, n2h = 0xFFu;
        raw_issue(ys - 2 * d);
        raw_issue_to(ys - d, w2m, w2h, n2m, n2h);
        raw_finish(ys - 2 * d, gt, ft, nbt, st, bt);
        raw_finish_from(ys - d, w2m, w2h, n2m, n2h, gt, ft, nbt, st, bt);
        raw_issue(ys);
        raw_issue_to(ys + d, w2m, w2h, n2m, n2h);
        raw_finish(ys, gA, fA, nbA, sA, bA);
        f_issue(ys, nbA);
        raw_finish_from(ys + d, w2m, w2h, n2m, n2h, gB, fB, nbB, sB, bB);
    } else if constexpr (!F::gstate && G1 && M == 0) {
        // FP64 / FP32: the first four ring rows two at a time, as above
        GWords<S> a1, a2, b1, b2;
        uint32_t na1, na2, nb1, nb2;
        real st, bt;
        g_row_issue(ys - 2 * d, a1, a2, na1, na2);
        g_row_issue(ys - d, b1, b2, nb1, nb2);
        g_row_finish(ys - 2 * d, a1, a2, na1, na2, st, bt);
        g_row_finish(ys - d, b1, b2, nb1, nb2, st, bt);
        g_row_issue(ys, a1, a2, na1, na2);
        g_row_issue(ys + d, b1, b2, nb1, nb2);
        g_row_finish(ys, a1, a2, na1, na2, sA, bA);
        nbA = na1;
        g_row_finish(ys + d, b1, b2, nb1, nb2, sB, bB);
        nbB = nb1;
    } else {
        {
            real gt[9], ft[9], st, bt;
            uint32_t nbt;
            fill_row(ys - 2 * d, gt, ft, nbt, st, bt);
            if constexpr (F::gstate) __syncthreads();
            fill_row(ys - d, gt, ft, nbt, st, bt);
            if constexpr (F::gstate) __syncthreads();
        }
        fill_row(ys, gA, fA, nbA, sA, bA);
        if constexpr (F::gstate) __syncthreads();
        fill_row(ys + d, gB, fB, nbB, sB, bB);
        if constexpr (F::gstate) __syncthreads();
        f_issue(ys, nbA);
    }
    raw_issue(ys + 2 * d);
    // Unrolled by three so the three rows of pulled values rotate roles
    // without copies (the last argument: the mask of the next row).
    for (int k = 0; k < nrow; k += 3) {
        step(ys + k * d, gA, fA, nbA, sA, bA, gC, fC, nbC, sC, bC, nbB);
        if (k + 1 >= nrow) break;
        step(ys + (k + 1) * d, gB, fB, nbB, sB, bB, gA, fA, nbA, sA, bA, nbC);
        if (k + 2 >= nrow) break;
        step(ys + (k + 2) * d, gC, fC, nbC, sC, bC, gB, fB, nbB, sB, bB, nbA);
    }

    if constexpr (DIAG) {
        // Wavefront reduction, then across the BX/64 wavefronts in a fixed order.
        __shared__ double red[BX / 64][5];
        double vals[5] = {d_drho, d_phi, d_ke, d_umax, d_n};
#pragma unroll
        for (int k = 0; k < 5; ++k) {
            double a = vals[k];
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) {
                const double b = __shfl_xor(a, off, 64);
                if (k == 3)
                    a = (b > a || b != b) ? b : a;
                else
                    a += b;
            }
            vals[k] = a;
        }
        const int lane = t & 63, wv = t >> 6;
        __syncthreads();
        if (lane == 0) {
#pragma unroll
            for (int k = 0; k < 5; ++k) red[wv][k] = vals[k];
        }
        __syncthreads();
        if (t == 0) {
            double o[5] = {0, 0, 0, 0, 0};
            for (int w = 0; w < BX / 64; ++w) {
                o[0] += red[w][0];
                o[1] += red[w][1];
                o[2] += red[w][2];
                o[3] = (red[w][3] > o[3] || red[w][3] != red[w][3]) ? red[w][3] : o[3];
                o[4] += red[w][4];
            }
            double* out = partials + (int64_t)tile_id * kPartials;
            out[0] = o[0] + o[4] * v.rho_ref;  // sum rho = n rho_ref + sum (rho - rho_ref)
            out[1] = o[1];
            out[2] = o[2];
            out[3] = o[3];
            out[4] = o[4];
            out[5] = 0.0;
        }
    }
}

// One step: workgroup b sweeps one tile. A single lattice takes logical tile
// xcd_tile(b, n) of its (grid_x x strips) tiling; a batch reads its tile table
// (already in XCD-aware order).
template <int S, int COLL, int BX, bool DIAG, bool G1, int M>
__global__ __launch_bounds__(BX) __attribute__((amdgpu_waves_per_eu(kWaves<S>)))
void sweep_kernel(const View* __restrict__ views, const Tile* __restrict__ tiles, int rows,
                  int grid_x, int parity, double* __restrict__ partials) {
    if (tiles) {
        const Tile tl = tiles[blockIdx.x];
        if (tl.member < 0) return;  // padding of a batch table (whole workgroup)
        sweep_tile<S, COLL, BX, DIAG, G1, M>(views, tl.member, tl.tx, tl.ty, tl.y0, tl.y1, tl.id,
                                             parity, partials);
    } else {
        const int tile_id = xcd_tile((int)blockIdx.x, (int)gridDim.x);
        const int tx = tile_id % grid_x, ty = tile_id / grid_x;
        sweep_tile<S, COLL, BX, DIAG, G1, M>(views, 0, tx, ty, ty * rows, ty * rows + rows,
                                             tile_id, parity, partials);
    }
}

// Persistent form of a window of `steps` timesteps of a batch: each workgroup
// takes work items in order from a counter, item i being tile i % n of step
// i / n (step-major, the tiles of a step in the table's order), and sweeps it
// once the tiles it depends on have finished the previous step. A tile's step
// reads the previous step's populations of its own tile and of the tiles
// holding nodes within three of it (the pulls and the phi stencil with its
// ghosts), and overwrites the buffer those tiles read in the previous step, so
// both hazards are covered by the same condition: done[d] >= step for every d
// listed in deps (kPersistDeps entries per tile, -1 = none, the tile itself
// included). There is no barrier between members or between steps.
//
// Progress: items are claimed in order and each depends only on items of the
// previous step, all claimed earlier by running workgroups, so the unfinished
// item of lowest step can always proceed; no workgroup waits on one that has
// not started. Every wait is bounded: after spin_limit polls or about one
// second (or once another workgroup has reported a timeout) the workgroup sets
// *err and leaves, so the grid always drains; the host reports the error.
//
// Memory ordering: a tile's populations are written by all its threads; each
// wave waits for its stores to complete before the barrier, after which thread
// 0 makes them visible device-wide (other XCDs included) with one agent-scope
// release fence (an L2 write-back), waits for that write-back to complete,
// and publishes the step with an atomic store. A waiting thread polls done[]
// with relaxed agent-scope loads and then issues one agent-scope acquire
// fence; the barrier that follows orders the tile's pulls after it.
constexpr uint64_t kWaitTicks = 100000000;  // one second of the 100 MHz wall clock
template <int S, int COLL, int BX, bool G1>
__global__ __launch_bounds__(BX) __attribute__((amdgpu_waves_per_eu(kWaves<S>)))
void sweep_persistent_kernel(const View* __restrict__ views, const Tile* __restrict__ tiles,
                             const int32_t* __restrict__ deps, int n_tiles, int steps,
                             int parity0, int32_t* done, uint32_t* next, int32_t* err,
                             uint32_t spin_limit) {
    __shared__ int s_item, s_abort;
    const int t = threadIdx.x;
    const int total = n_tiles * steps;
    // Thread 0 publishes the previous item's step (after the barrier that ends
    // it) in the same block as the next claim, so each iteration has one
    // thread-0 block at its top, then barriers and branches that are uniform.
    int prev_j = -1, prev_k = 0;
    for (;;) {
        if (t == 0) {
            // relaxed: thread 0's release fence at the end of the item orders it
            if (prev_j >= 0)
                __hip_atomic_store(done + prev_j, prev_k + 1, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
            s_item = (int)atomicAdd(next, 1u);
            s_abort = 0;
        }
        __syncthreads();
        // Uniform values read through readfirstlane, so that the compiler
        // treats the loop exits as uniform.
        const int item = __builtin_amdgcn_readfirstlane(s_item);
        if (item >= total) break;
        const int k = item / n_tiles, j = item - k * n_tiles;
        if (t < kPersistDeps) {
            const int d = deps[(int64_t)j * kPersistDeps + t];
            if (d >= 0 &&
                __hip_atomic_load(done + d, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < k) {
                // Poll with relaxed loads (no cache invalidation per poll); the
                // acquire fence after the loop orders the tile's reads. Bounded
                // by spin_limit polls and by about one second of wall clock.
                const uint64_t t0 = (uint64_t)wall_clock64();
                uint32_t polls = 0;
                while (__hip_atomic_load(done + d, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < k) {
                    if (++polls > spin_limit || (uint64_t)wall_clock64() - t0 > kWaitTicks ||
                        __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
                        __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        s_abort = 1;
                        break;
                    }
                    __builtin_amdgcn_s_sleep(2);
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        }
        __syncthreads();
        if (__builtin_amdgcn_readfirstlane(s_abort)) break;
        const Tile tl = tiles[j];
        sweep_tile<S, COLL, BX, false, G1, 0>(views, tl.member, tl.tx, tl.ty, tl.y0, tl.y1, tl.id,
                                              (parity0 + k) & 1, nullptr);
        // Every wave waits until its stores have completed (reached L2), then
        // the barrier; thread 0's agent-scope release (one L2 write-back for the
        // workgroup) then covers the whole tile when it publishes the step. The
        // explicit wait keeps the publication behind the completed write-back.
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        if (t == 0) {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            __builtin_amdgcn_s_waitcnt(0);
        }
        prev_j = j;
        prev_k = k;
    }
    if (t == 0 && prev_j >= 0)
        __hip_atomic_store(done + prev_j, prev_k + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// In-place pre-pass: phi of S_n at the tile-border nodes, into View::band,
// with the arithmetic of the sweep's own phi (the same pulls summed in the same
// order, so the sweep obtains the same bits either way). The nodes are the rows
// y0, y0+1, y1-2, y1-1 of every strip [y0, y1) of `rows` rows (full width) and
// the columns x0, x0+1, x1-2, x1-1 of every tile column [x0, x1) of `bx`
// columns (every row): the rows beyond the ends of a strip and the halo
// columns of a tile for its neighbours, two deep (the stencil and the ghost
// values at solid nodes). Solid nodes get 0. Rows or columns counted twice on
// small lattices are written twice with the same value.
// Each wavefront takes 64 nodes of one row (waves 0 .. row_waves-1: band row
// w / xchunks, columns 64 (w % xchunks) + lane; then row (w - row_waves) /
// cchunks, band columns 64 ((w - row_waves) % cchunks) + lane), so the row, and
// with it the buffer descriptors, is uniform across the wavefront.
template <int S, int M, bool G1>
__global__ __launch_bounds__(256) void band_kernel(const View* __restrict__ views, int bx,
                                                   int rows, int row_waves, int xchunks,
                                                   int cchunks, int cols_per_row) {
    using F = Fmt<S>;
    using real = typename F::real;
    const View v = views[0];
    const int nx = v.nx, ny = v.ny;
    const int lane = (int)(threadIdx.x & 63);
    const int w = __builtin_amdgcn_readfirstlane((int)(blockIdx.x * 4 + (threadIdx.x >> 6)));
    int x, y;
    if (w < row_waves) {
        const int j = w / xchunks, ch = w - j * xchunks;
        const int k = j & 3;
        const int y0 = (j >> 2) * rows, y1 = min(y0 + rows, ny);
        y = wrap(k < 2 ? y0 + k : y1 - 4 + k, ny);
        x = ch * 64 + lane;
        if (x >= nx) return;
    } else {
        const int w2 = w - row_waves;
        y = w2 / cchunks;
        if (y >= ny) return;
        const int j = (w2 - y * cchunks) * 64 + lane;
        if (j >= cols_per_row) return;
        const int k = j & 3;
        const int x0 = (j >> 2) * bx, x1 = min(x0 + bx, nx);
        x = wrap(k < 2 ? x0 + k : x1 - 4 + k, nx);
    }
    const size_t node = (size_t)y * v.pitch + x;
    const uint32_t nb = v.nbr[node];
    real ph = 0;
    if (nb != 0xFFu) {
        const uint32_t xm = x == 0 ? nx - 1 : x - 1, xp = x == nx - 1 ? 0 : x + 1;
        const Rows R = rows_of(v.buf[0], v, y, wrap(y - 1, ny), wrap(y + 1, ny));
        const ColOff co = col_offsets<S>((uint32_t)x, xm, xp);
        real small = 0, base = 0;
        if constexpr (G1) {
            ph = phi9<S, M>(R, v, co, nb, small, base);
        } else {
            real g[9];
            pull9<S, 9, M>(R, v, co, nb, g, &base);
#pragma unroll
            for (int i = 0; i < 9; ++i) small += g[i];
            ph = base + small;
        }
    }
    reinterpret_cast<real*>(v.band)[node] = ph;
}

// Lattice-node bounce-back (Fig. 9b), the wall nodes' part of a step: every
// solid node with fluid neighbours sends back along each link to a fluid
// neighbour what that neighbour sent it in the previous step (the post-
// collision f_j, g_j of r = w - e_j, read from the source buffer), storing it
// at w in plane OPP(j) of the destination buffer, where r pulls it in the next
// step. Only wall-node slots are written, so this launch and the sweep of the
// same step are independent. Tiles as in the sweep; each thread scans one
// column of its tile.
template <int S>
__global__ __launch_bounds__(1024) void wall_kernel(const View* __restrict__ views,
                                                   const Tile* __restrict__ tiles, int rows,
                                                   int grid_x, int parity) {
    int member = 0, tx, y0, y1;
    if (tiles) {
        const Tile tl = tiles[blockIdx.x];
        if (tl.member < 0) return;  // padding of a batch table
        member = tl.member;
        tx = tl.tx;
        y0 = tl.y0;
        y1 = tl.y1;
    } else {
        tx = (int)blockIdx.x % grid_x;
        y0 = ((int)blockIdx.x / grid_x) * rows;
        y1 = y0 + rows;
    }
    const View v = views[member];
    if (!v.bounce) return;
    const int nx = v.nx, ny = v.ny;
    const int x = tx * (int)blockDim.x + (int)threadIdx.x;
    if (x >= nx) return;
    const char* src = parity ? v.buf[1] : v.buf[0];
    char* dst = parity ? v.buf[0] : v.buf[1];
    const uint32_t xm = x == 0 ? nx - 1 : x - 1, xp = x == nx - 1 ? 0 : x + 1;
    const ColOff co = col_offsets<S>((uint32_t)x, xm, xp);
    y1 = min(y1, ny);
    for (int y = y0; y < y1; ++y) {
        const size_t node = (size_t)y * v.pitch + x;
        if (v.nbr[node] != 0xFFu) continue;
        const uint32_t fl = v.grec[node];  // bit m-1: w + e_m is fluid
        if (fl == 0u) continue;
        const Rows R = rows_of(src, v, y, wrap(y - 1, ny), wrap(y + 1, ny));
        const Rsrc out = row_rsrc(dst, v, y);
        static_for<8>([&](auto jc) {
            constexpr int j = decltype(jc)::value + 1;
            if ((fl >> (OPP[j] - 1)) & 1u) {  // the source w - e_j is fluid
                constexpr int r = src_row<0, j>(), c = src_col<0, j>();
                stp<S, OPP[j]>(out, v, co, ldp<S, j>(R.r[r], v, co, c));
                stp<S, 9 + OPP[j]>(out, v, co, ldp<S, 9 + j>(R.r[r], v, co, c));
            }
        });
    }
}

// ------------------------------------------------------------------ sweep launchers
// The sweep and band kernels of one storage format are instantiated by
// sweep_fmt<S> / band_fmt<S>; the build compiles this file once per format with
// LB_SWEEP_UNIT = S (those instantiations only) and once without it (every
// other kernel), so the formats compile in parallel.

struct SweepArgs {
    int collision, block_x;
    bool diag, tau_phi_one, inplace;
    const View* views;
    const Tile* tiles;
    int n1d, gx, gy, rows, parity;
    double* partials;
    hipStream_t stream;
};

template <int S, int C, int BX, bool D, bool G1>
static hipError_t sweep_one(const SweepArgs& a) {
    const dim3 grid = a.tiles ? dim3(a.n1d) : dim3(a.gx * a.gy);
    if constexpr (S == ST_F64 || S == ST_F32) {
        if (a.inplace) {
            if (a.parity)
                hipLaunchKernelGGL((sweep_kernel<S, C, BX, D, G1, 2>), grid, dim3(BX), 0, a.stream,
                                   a.views, a.tiles, a.rows, a.gx, a.parity, a.partials);
            else
                hipLaunchKernelGGL((sweep_kernel<S, C, BX, D, G1, 1>), grid, dim3(BX), 0, a.stream,
                                   a.views, a.tiles, a.rows, a.gx, a.parity, a.partials);
            return hipGetLastError();
        }
    }
    hipLaunchKernelGGL((sweep_kernel<S, C, BX, D, G1, 0>), grid, dim3(BX), 0, a.stream, a.views,
                       a.tiles, a.rows, a.gx, a.parity, a.partials);
    return hipGetLastError();
}

template <int S, int C, int BX, bool D>
static hipError_t sweep_g(const SweepArgs& a) {
    if constexpr (Fmt<S>::gstate)  // the compressed formats exist only for tau_phi = 1
        return sweep_one<S, C, BX, D, true>(a);
    return a.tau_phi_one ? sweep_one<S, C, BX, D, true>(a) : sweep_one<S, C, BX, D, false>(a);
}

template <int S, int C, int BX>
static hipError_t sweep_d(const SweepArgs& a) {
    return a.diag ? sweep_g<S, C, BX, true>(a) : sweep_g<S, C, BX, false>(a);
}

template <int S, int C>
static hipError_t sweep_b(const SweepArgs& a) {
    switch (a.block_x) {
        case 64: return sweep_d<S, C, 64>(a);
        case 128: return sweep_d<S, C, 128>(a);
        case 256: return sweep_d<S, C, 256>(a);
        case 512: return sweep_d<S, C, 512>(a);
        case 1024:  // the F64C rings in LDS do not fit 1024 columns
            if constexpr (S != ST_F64C) return sweep_d<S, C, 1024>(a);
            else return hipErrorInvalidValue;
        default: return hipErrorInvalidValue;
    }
}

struct PersistArgs {
    int collision, block_x;
    bool tau_phi_one;
    const View* views;
    const Tile* tiles;
    const int32_t* deps;
    int n_tiles, steps, parity0, grid;
    int32_t* done;
    uint32_t* next;
    int32_t* err;
    uint32_t spin_limit;
    hipStream_t stream;
};

template <int S, int C, int BX>
static hipError_t persist_g(const PersistArgs& a) {
    auto go = [&](auto kernel) {
        hipLaunchKernelGGL(kernel, dim3(a.grid), dim3(BX), 0, a.stream, a.views, a.tiles, a.deps,
                           a.n_tiles, a.steps, a.parity0, a.done, a.next, a.err, a.spin_limit);
    };
    if (Fmt<S>::gstate || a.tau_phi_one) go(sweep_persistent_kernel<S, C, BX, true>);
    else if constexpr (!Fmt<S>::gstate) go(sweep_persistent_kernel<S, C, BX, false>);
    return hipGetLastError();
}

template <int S, int C>
static hipError_t persist_b(const PersistArgs& a) {
    switch (a.block_x) {
        case 128: return persist_g<S, C, 128>(a);
        case 256: return persist_g<S, C, 256>(a);
        case 512: return persist_g<S, C, 512>(a);
        default: return hipErrorInvalidValue;
    }
}

template <int S>
hipError_t persist_fmt(const PersistArgs& a) {
    return a.collision == CO_MRT ? persist_b<S, CO_MRT>(a) : persist_b<S, CO_BGK>(a);
}

// Workgroups of the persistent kernel that fit on the device at once.
template <int S>
hipError_t persist_occupancy(int block_x, int collision, bool tau_phi_one, int* per_cu) {
    hipError_t e = hipErrorInvalidValue;
    auto occ = [&](auto kernel, int bx) {
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, kernel, bx, 0);
    };
    const bool g1 = Fmt<S>::gstate || tau_phi_one;
#define LB_OCC(C, BX)                                                                   \
    if (g1) occ(sweep_persistent_kernel<S, C, BX, true>, BX);                           \
    else if constexpr (!Fmt<S>::gstate) occ(sweep_persistent_kernel<S, C, BX, false>, BX);
    if (collision == CO_MRT) {
        if (block_x == 128) { LB_OCC(CO_MRT, 128) }
        else if (block_x == 256) { LB_OCC(CO_MRT, 256) }
        else if (block_x == 512) { LB_OCC(CO_MRT, 512) }
    } else {
        if (block_x == 128) { LB_OCC(CO_BGK, 128) }
        else if (block_x == 256) { LB_OCC(CO_BGK, 256) }
        else if (block_x == 512) { LB_OCC(CO_BGK, 512) }
    }
#undef LB_OCC
    return e;
}

template <int S>
hipError_t sweep_fmt(const SweepArgs& a) {
    if (a.inplace && (a.tiles || (S != ST_F64 && S != ST_F32))) return hipErrorInvalidValue;
    return a.collision == CO_MRT ? sweep_b<S, CO_MRT>(a) : sweep_b<S, CO_BGK>(a);
}

struct BandArgs {
    int bx, rows, row_waves, xchunks, cchunks, cols_per_row;
};

template <int S>
hipError_t band_fmt(bool g1, int parity, dim3 grid, const View* v, BandArgs b, hipStream_t st) {
    if constexpr (S == ST_F64 || S == ST_F32) {
        auto go = [&](auto kernel) {
            hipLaunchKernelGGL(kernel, grid, dim3(256), 0, st, v, b.bx, b.rows, b.row_waves,
                               b.xchunks, b.cchunks, b.cols_per_row);
        };
        if (parity) {
            if (g1) go(band_kernel<S, 2, true>);
            else go(band_kernel<S, 2, false>);
        } else {
            if (g1) go(band_kernel<S, 1, true>);
            else go(band_kernel<S, 1, false>);
        }
        return hipGetLastError();
    }
    return hipErrorInvalidValue;
}

template <int S>
hipError_t wall_fmt(const SweepArgs& a) {
    if constexpr (S == ST_F64 || S == ST_F32) {
        const dim3 grid = a.tiles ? dim3(a.n1d) : dim3(a.gx * a.gy);
        hipLaunchKernelGGL((wall_kernel<S>), grid, dim3(a.block_x), 0, a.stream, a.views, a.tiles,
                           a.rows, a.gx, a.parity);
        return hipGetLastError();
    }
    return hipErrorInvalidValue;
}

#ifdef LB_SWEEP_UNIT
template hipError_t sweep_fmt<LB_SWEEP_UNIT>(const SweepArgs&);
template hipError_t persist_fmt<LB_SWEEP_UNIT>(const PersistArgs&);
template hipError_t persist_occupancy<LB_SWEEP_UNIT>(int, int, bool, int*);
template hipError_t wall_fmt<LB_SWEEP_UNIT>(const SweepArgs&);
template hipError_t band_fmt<LB_SWEEP_UNIT>(bool, int, dim3, const View*, BandArgs, hipStream_t);
#else
#define LB_EXTERN_FMT(S)                                                                   \
    extern template hipError_t sweep_fmt<S>(const SweepArgs&);                             \
    extern template hipError_t persist_fmt<S>(const PersistArgs&);                         \
    extern template hipError_t persist_occupancy<S>(int, int, bool, int*);                 \
    extern template hipError_t wall_fmt<S>(const SweepArgs&);                              \
    extern template hipError_t band_fmt<S>(bool, int, dim3, const View*, BandArgs, hipStream_t);
LB_EXTERN_FMT(ST_F64)
LB_EXTERN_FMT(ST_F32)
LB_EXTERN_FMT(ST_F16S)
LB_EXTERN_FMT(ST_BF16S)
LB_EXTERN_FMT(ST_F64C)
LB_EXTERN_FMT(ST_F32C)
#undef LB_EXTERN_FMT

hipError_t launch_sweep(int storage, int collision, int block_x, bool diag, bool tau_phi_one,
                        bool inplace, const View* d_views, const Tile* d_tiles, int n_blocks_1d,
                        int grid_x, int grid_y, int rows, int parity, double* partials,
                        hipStream_t stream) {
    const SweepArgs a{collision, block_x, diag, tau_phi_one, inplace, d_views, d_tiles,
                      n_blocks_1d, grid_x, grid_y, rows, parity, partials, stream};
    switch (storage) {
        case ST_F64: return sweep_fmt<ST_F64>(a);
        case ST_F32: return sweep_fmt<ST_F32>(a);
        case ST_F16S: return sweep_fmt<ST_F16S>(a);
        case ST_BF16S: return sweep_fmt<ST_BF16S>(a);
        case ST_F64C: return sweep_fmt<ST_F64C>(a);
        case ST_F32C: return sweep_fmt<ST_F32C>(a);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_persistent(int storage, int collision, int block_x, bool tau_phi_one,
                             const View* d_views, const Tile* d_tiles, const int32_t* d_deps,
                             int n_tiles, int steps, int parity0, int grid, int32_t* done,
                             uint32_t* next, int32_t* err, uint32_t spin_limit,
                             hipStream_t stream) {
    if (n_tiles < 1 || steps < 1 || grid < 1 || (int64_t)n_tiles * steps >= ((int64_t)1 << 31))
        return hipErrorInvalidValue;
    const PersistArgs a{collision, block_x, tau_phi_one, d_views, d_tiles, d_deps, n_tiles,
                        steps, parity0, grid, done, next, err, spin_limit, stream};
    switch (storage) {
        case ST_F64: return persist_fmt<ST_F64>(a);
        case ST_F32: return persist_fmt<ST_F32>(a);
        case ST_F16S: return persist_fmt<ST_F16S>(a);
        case ST_BF16S: return persist_fmt<ST_BF16S>(a);
        case ST_F64C: return persist_fmt<ST_F64C>(a);
        case ST_F32C: return persist_fmt<ST_F32C>(a);
        default: return hipErrorInvalidValue;
    }
}

hipError_t persistent_occupancy(int storage, int collision, int block_x, bool tau_phi_one,
                                int* per_cu) {
    switch (storage) {
        case ST_F64: return persist_occupancy<ST_F64>(block_x, collision, tau_phi_one, per_cu);
        case ST_F32: return persist_occupancy<ST_F32>(block_x, collision, tau_phi_one, per_cu);
        case ST_F16S: return persist_occupancy<ST_F16S>(block_x, collision, tau_phi_one, per_cu);
        case ST_BF16S: return persist_occupancy<ST_BF16S>(block_x, collision, tau_phi_one, per_cu);
        case ST_F64C: return persist_occupancy<ST_F64C>(block_x, collision, tau_phi_one, per_cu);
        case ST_F32C: return persist_occupancy<ST_F32C>(block_x, collision, tau_phi_one, per_cu);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_walls(int storage, int block_x, const View* d_views, const Tile* d_tiles,
                        int n_blocks_1d, int grid_x, int grid_y, int rows, int parity,
                        hipStream_t stream) {
    if (block_x < 1 || block_x > 1024 || rows < 1) return hipErrorInvalidValue;
    const SweepArgs a{0, block_x, false, false, false, d_views, d_tiles,
                      n_blocks_1d, grid_x, grid_y, rows, parity, nullptr, stream};
    if (storage == ST_F64) return wall_fmt<ST_F64>(a);
    if (storage == ST_F32) return wall_fmt<ST_F32>(a);
    return hipErrorInvalidValue;
}

hipError_t launch_band(int storage, bool tau_phi_one, const View* d_view, int nx, int ny,
                       int block_x, int rows, int parity, hipStream_t stream) {
    if (block_x < 1 || rows < 1) return hipErrorInvalidValue;
    const int64_t strips = (ny + rows - 1) / rows, tiles_x = (nx + block_x - 1) / block_x;
    BandArgs b;
    b.bx = block_x;
    b.rows = rows;
    b.xchunks = (nx + 63) / 64;
    b.cols_per_row = (int)(4 * tiles_x);
    b.cchunks = (b.cols_per_row + 63) / 64;
    const int64_t row_waves = 4 * strips * b.xchunks;
    const int64_t waves = row_waves + (int64_t)ny * b.cchunks;
    if (waves >= ((int64_t)1 << 31)) return hipErrorInvalidValue;
    b.row_waves = (int)row_waves;
    const dim3 grid((unsigned)((waves + 3) / 4));
    if (storage == ST_F64) return band_fmt<ST_F64>(tau_phi_one, parity, grid, d_view, b, stream);
    if (storage == ST_F32) return band_fmt<ST_F32>(tau_phi_one, parity, grid, d_view, b, stream);
    return hipErrorInvalidValue;
}

// Sum per-workgroup partial records in a fixed order: one workgroup per member.
__global__ __launch_bounds__(256) void finalize_kernel(const int32_t* __restrict__ member_first,
                                                       int n_records_single,
                                                       const double* __restrict__ partials,
                                                       double* __restrict__ diag_out,
                                                       int32_t* __restrict__ flag) {
    const int m = blockIdx.x;
    const int first = member_first ? member_first[m] : 0;
    const int last = member_first ? member_first[m + 1] : n_records_single;
    __shared__ double red[256][6];
    double a[6] = {0, 0, 0, 0, 0, 0};
    for (int r = first + (int)threadIdx.x; r < last; r += 256) {
        const double* p = partials + (int64_t)r * kPartials;
        a[0] += p[0];
        a[1] += p[1];
        a[2] += p[2];
        a[3] = (p[3] > a[3] || p[3] != p[3]) ? p[3] : a[3];
        a[4] += p[4];
        a[5] += p[5];
    }
#pragma unroll
    for (int k = 0; k < 6; ++k) red[threadIdx.x][k] = a[k];
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            double* x = red[threadIdx.x];
            const double* y = red[threadIdx.x + s];
            x[0] += y[0];
            x[1] += y[1];
            x[2] += y[2];
            x[3] = (y[3] > x[3] || y[3] != y[3]) ? y[3] : x[3];
            x[4] += y[4];
            x[5] += y[5];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        double* o = diag_out + (int64_t)m * kPartials;
#pragma unroll
        for (int k = 0; k < 6; ++k) o[k] = red[0][k];
        const bool bad = !isfinite(red[0][0]) || !isfinite(red[0][1]) || !isfinite(red[0][2]) ||
                         !(red[0][3] == red[0][3]);
        if (bad) flag[m] = 1;
    }
}

// ------------------------------------------------------------------ helpers for
// the non-hot kernels: absolute FP64 values of a node's pulled populations.

__device__ inline double rest_f(const View& v, int i) {
    if (v.storage == ST_F64 || v.storage == ST_F64C) return 0.0;
    return i == 0 ? v.rho_ref - 5.0 / 3.0 * v.p0_ref : (i < 5 ? 1.0 / 3.0 : 1.0 / 12.0) * v.p0_ref;
}

template <int S>
__device__ inline bool pull_node_abs(const View& v, int parity, int x, int y, double f[9],
                                     double g[9]) {
    const int nx = v.nx, ny = v.ny;
    const uint32_t nb = v.nbr[(size_t)y * v.pitch + x];
    if (nb == 0xFFu) return false;
    const char* src = parity ? v.buf[1] : v.buf[0];
    typename Fmt<S>::real a[9], b[9], base;
    const uint32_t xm = x == 0 ? nx - 1 : x - 1, xp = x == nx - 1 ? 0 : x + 1;
    const Rows R = rows_of(src, v, y, wrap(y - 1, ny), wrap(y + 1, ny));
    const ColOff co = col_offsets<S>((uint32_t)x, xm, xp);
    if constexpr (S == ST_F64 || S == ST_F32) {
        if (v.inplace) {
            if (parity) {
                pull9<S, 0, 2>(R, v, co, nb, a);
                pull9<S, 9, 2>(R, v, co, nb, b, &base);
            } else {
                pull9<S, 0, 1>(R, v, co, nb, a);
                pull9<S, 9, 1>(R, v, co, nb, b, &base);
            }
            for (int i = 0; i < 9; ++i) {
                f[i] = (double)a[i] + rest_f(v, i);
                g[i] = (double)b[i];
            }
            g[0] += (double)base;
            return true;
        }
    }
    const uint32_t nbp = ((S == ST_F64 || S == ST_F32) && v.bounce) ? 0u : nb;
    pull9<S, 0>(R, v, co, nbp, a);
    if constexpr (Fmt<S>::gstate) {
        // g of S_n from the stored g-state: g_i = g^eq_i of r - e_i (or of r in
        // the opposite direction across a solid link), g_0 = phi - sum g^eq_i.
        using Rl = typename Fmt<S>::real;
        using E = typename Fmt<S>::template E<10>;
        auto st = [&](const Rsrc& rr, uint32_t xx, Rl& ph, Rl& gm, Rl& gu, Rl& gv, double& pa) {
            if constexpr (S == ST_F32C) {
                const uint32_t u = buf_ld<uint32_t>(rr, xx * 4, Fmt<S>::template poff<9>(v));
                ph = G0Code::b(u) + G0Code::q(u);
                pa = (double)G0Code::b(u) + (double)G0Code::q(u);
            } else {
                ph = buf_ld<E>(rr, xx * sizeof(E), Fmt<S>::template poff<9>(v));
                pa = ph;
            }
            gm = buf_ld<E>(rr, xx * sizeof(E), Fmt<S>::template poff<10>(v));
            gu = buf_ld<E>(rr, xx * sizeof(E), Fmt<S>::template poff<11>(v));
            gv = buf_ld<E>(rr, xx * sizeof(E), Fmt<S>::template poff<12>(v));
        };
        Rl ph0, gm0, gu0, gv0;
        double pa0;
        st(R.r[0], (uint32_t)x, ph0, gm0, gu0, gv0, pa0);
        double out = 0;
        static_for<9>([&](auto ic) {
            constexpr int i = decltype(ic)::value;
            if constexpr (i > 0) {
                out += (double)geq_dir<i>(ph0, gm0, gu0, gv0);
                if ((nb >> (i - 1)) & 1u) {
                    b[i] = geq_dir<OPP[i]>(ph0, gm0, gu0, gv0);
                } else {
                    constexpr int r = EY[i] > 0 ? 1 : (EY[i] < 0 ? 2 : 0);
                    const uint32_t xx = EX[i] > 0 ? xm : (EX[i] < 0 ? xp : (uint32_t)x);
                    Rl ph1, gm1, gu1, gv1;
                    double pa1;
                    st(R.r[r], xx, ph1, gm1, gu1, gv1, pa1);
                    b[i] = geq_dir<i>(ph1, gm1, gu1, gv1);
                }
            }
        });
        for (int i = 0; i < 9; ++i) f[i] = (double)a[i] + rest_f(v, i);
        g[0] = pa0 - out;
        for (int i = 1; i < 9; ++i) g[i] = (double)b[i];
        return true;
    }
    pull9<S, 9>(R, v, co, nbp, b, &base);
    for (int i = 0; i < 9; ++i) {
        f[i] = (double)a[i] + rest_f(v, i);
        g[i] = (double)b[i];
    }
    g[0] += (double)base;  // exact: G0Code keeps g_0 = base + q
    return true;
}

// ------------------------------------------------------------------ initial state

// S_0 = equilibria of the initial fields (ghost phi at solid nodes, stencils of
// Eq. (best), Appendix A with the initial velocity), arithmetic in FP64, then
// "un-streamed" into buf[0] so that the first pull of the sweep yields S_0:
// the population S_0 f_i(r) is stored at the node it would have left, r - e_i,
// or, across a solid link, at r in the opposite direction.
template <int S>
__global__ __launch_bounds__(256) void init_kernel(View v, const double* __restrict__ phi0,
                                                   const double* __restrict__ rho0,
                                                   const double* __restrict__ ux0,
                                                   const double* __restrict__ uy0) {
    const int64_t n = (int64_t)v.nx * v.ny;
    const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= n) return;
    const int x = (int)(id % v.nx), y = (int)(id / v.nx);
    const int nx = v.nx, ny = v.ny, pitch = v.pitch;
    const int64_t r = (int64_t)y * pitch + x;
    const uint32_t nb = v.nbr[r];
    // In place, rho0, ux0, uy0 are staged in the node's own slots of planes
    // 1..3 (FP64) or 1..6 (FP32, low and high words), which only this thread
    // reads and then overwrites (layout P keeps every value at its node).
    constexpr int kEs = sizeof(typename Fmt<S>::template E<2>);
    const Rsrc own = row_rsrc(v.buf[0], v, y);
    auto staged = [&](int q) -> double {
        if constexpr (kEs == 8) {
            return buf_ld<double>(own, (uint32_t)x * 8, (1 + q) * pitch * 8);
        } else {
            const uint64_t lo = buf_ld<uint32_t>(own, (uint32_t)x * 4, (1 + 2 * q) * pitch * 4);
            const uint64_t hi = buf_ld<uint32_t>(own, (uint32_t)x * 4, (2 + 2 * q) * pitch * 4);
            return __builtin_bit_cast(double, lo | (hi << 32));
        }
    };
    if (nb == 0xFFu) {
        if (v.inplace)
            for (int pl = 1; pl <= (kEs == 8 ? 3 : 6); ++pl) {
                if constexpr (kEs == 8) buf_st<double>(0.0, own, (uint32_t)x * 8, pl * pitch * 8);
                else buf_st<uint32_t>(0u, own, (uint32_t)x * 4, pl * pitch * 4);
            }
        return;
    }
    auto host_idx = [&](int xx, int yy) { return (int64_t)wrap(yy, ny) * nx + wrap(xx, nx); };
    auto dev_idx = [&](int xx, int yy) { return (int64_t)wrap(yy, ny) * pitch + wrap(xx, nx); };
    auto phi_at = [&](int xx, int yy) -> double {
        const int64_t s = dev_idx(xx, yy);
        if (v.nbr[s] != 0xFFu) return phi0[host_idx(xx, yy)];
        const uint32_t rec = v.grec[s];
        const double dw = (S == ST_F64 || S == ST_F64C) ? reinterpret_cast<const double*>(v.dphi)[s]
                                      : (double)reinterpret_cast<const float*>(v.dphi)[s];
        const uint32_t axis = rec & 0xFu;
        const uint32_t bits = axis ? axis : (rec >> 4);
        const int m0 = axis ? 1 : 5;
        double sum = 0;
        int cnt = 0;
        for (int mm = 0; mm < 4; ++mm)
            if ((bits >> mm) & 1u) {
                sum += phi0[host_idx(xx + EX[m0 + mm], yy + EY[m0 + mm])];
                ++cnt;
            }
        if (cnt == 0) return 0.0;
        return sum / cnt - (axis ? dw : 1.4142135623730951 * dw);
    };
    double pn[9];
    for (int k = 0; k < 9; ++k) pn[k] = phi_at(x + EX[k], y + EY[k]);
    const double ph = pn[0];
    const double gx = (4.0 * (pn[1] - pn[2]) + (pn[5] - pn[7]) + (pn[8] - pn[6])) / 12.0;
    const double gy = (4.0 * (pn[3] - pn[4]) + (pn[5] - pn[8]) + (pn[7] - pn[6])) / 12.0;
    const double lap = (4.0 * (pn[1] + pn[2] + pn[3] + pn[4]) + (pn[5] + pn[6] + pn[7] + pn[8]) -
                        20.0 * ph) / 6.0;
    const int64_t hi = (int64_t)y * nx + x;
    const bool ip = (S == ST_F64 || S == ST_F32) && v.inplace;
    const double rho = ip ? staged(0) : rho0[hi];
    const double ux = ip ? staged(1) : ux0[hi];
    const double uy = ip ? staged(2) : uy0[hi];
    const double mu = ph * (v.A + v.B * ph * ph) - v.kappa * lap;
    const double p0 = rho / 3.0 + ph * ph * (0.5 * v.A + 0.75 * v.B * ph * ph);
    const double usq = ux * ux + uy * uy;
    double feq[9], geq[9], sf = 0, sg = 0;
    for (int i = 1; i < 9; ++i) {
        const double w = i < 5 ? 1.0 / 3.0 : 1.0 / 12.0;
        double wxx, wyy, wxy;
        if (i < 3) {
            wxx = 1.0 / 3.0; wyy = -1.0 / 6.0; wxy = 0;
        } else if (i < 5) {
            wxx = -1.0 / 6.0; wyy = 1.0 / 3.0; wxy = 0;
        } else {
            wxx = -1.0 / 24.0; wyy = -1.0 / 24.0; wxy = i < 7 ? 0.25 : -0.25;
        }
        const double eu = EX[i] * ux + EY[i] * uy;
        feq[i] = w * (p0 - v.kappa * ph * lap + rho * eu + 1.5 * rho * (eu * eu - usq / 3.0)) +
                 v.kappa * (wxx * gx * gx + wyy * gy * gy + wxy * gx * gy);
        geq[i] = w * (v.Gamma * mu + ph * eu + 1.5 * ph * (eu * eu - usq / 3.0));
        sf += feq[i];
        sg += geq[i];
    }
    feq[0] = rho - sf;
    geq[0] = ph - sg;
    char* dst = v.buf[0];
    using R = typename Fmt<S>::real;
    if constexpr (S == ST_F64 || S == ST_F32) {
        if (ip) {
            // layout P (the populations that have arrived at r, at r in plane
            // i), which the first step reads in phase 1: S_0 at r is the
            // equilibrium of r itself
            const ColOff co = col_offsets<S>((uint32_t)x, (uint32_t)x, (uint32_t)x);
            static_for<9>([&](auto ic) {
                constexpr int i = decltype(ic)::value;
                stp<S, i>(own, v, co, (R)(feq[i] - rest_f(v, i)));
                if constexpr (i == 0) {
                    if constexpr (Fmt<S>::shifted) {
                        const double b = geq[0] > 0.5 ? 1.0 : (geq[0] < -0.5 ? -1.0 : 0.0);
                        buf_st<uint32_t>(G0Code::enc((float)(geq[0] - b), (float)b), own, co.c9,
                                         Fmt<S>::template poff<9>(v));
                    } else {
                        stp<S, 9>(own, v, co, (R)geq[0]);
                    }
                } else {
                    stp<S, 9 + i>(own, v, co, (R)geq[i]);
                }
            });
            return;
        }
    }
    // Lattice-node bounce-back: no value waits across a solid link (the wall
    // node holds it), and the wall node's first pull finds what this node's
    // equilibrium sends into it, at r in the plane of that direction.
    bool lnode = false;
    if constexpr (S == ST_F64 || S == ST_F32) {
        lnode = v.bounce != 0;
        if (lnode) {
            const ColOff oco = col_offsets<S>((uint32_t)x, (uint32_t)x, (uint32_t)x);
            static_for<8>([&](auto jc) {
                constexpr int j = decltype(jc)::value + 1;
                if ((nb >> (OPP[j] - 1)) & 1u) {  // r + e_j is solid
                    stp<S, j>(own, v, oco, (R)(feq[j] - rest_f(v, j)));
                    stp<S, 9 + j>(own, v, oco, (R)geq[j]);
                }
            });
        }
    }
    static_for<9>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        const bool bb = !lnode && i > 0 && ((nb >> (i - 1)) & 1u);
        // Across a solid link the value waits at r in the opposite direction's plane.
        const int xs = bb ? x : wrap(x - EX[i], nx), ys = bb ? y : wrap(y - EY[i], ny);
        const Rsrc row = row_rsrc(dst, v, ys);
        const ColOff co = col_offsets<S>((uint32_t)xs, (uint32_t)xs, (uint32_t)xs);
        if constexpr (Fmt<S>::gstate) {
            // f as in the other formats; the g-state of S_0 is (phi_0, 0, 0, 0),
            // whose pulled g has the sum phi_0 (all the first collision uses)
            const int io = bb ? OPP[i] : i;
            const double fv = feq[i] - rest_f(v, io);
            if (bb) stp<S, OPP[i]>(row, v, co, (R)fv);
            else stp<S, i>(row, v, co, (R)fv);
            if constexpr (i == 0) {
                if constexpr (S == ST_F32C) {
                    const double b = ph > 0.5 ? 1.0 : (ph < -0.5 ? -1.0 : 0.0);
                    buf_st<uint32_t>(G0Code::enc((float)(ph - b), (float)b), row, co.c9,
                                     Fmt<S>::template poff<9>(v));
                } else {
                    stp<S, 9>(row, v, co, (R)ph);
                }
                stp<S, 10>(row, v, co, (R)0);
                stp<S, 11>(row, v, co, (R)0);
                stp<S, 12>(row, v, co, (R)0);
            }
        } else if constexpr (i == 0) {
            stp<S, 0>(row, v, co, (R)(feq[0] - rest_f(v, 0)));
            if constexpr (Fmt<S>::shifted) {
                const double b = geq[0] > 0.5 ? 1.0 : (geq[0] < -0.5 ? -1.0 : 0.0);
                buf_st<uint32_t>(G0Code::enc((float)(geq[0] - b), (float)b), row, co.c9,
                                 Fmt<S>::template poff<9>(v));
            } else {
                stp<S, 9>(row, v, co, (R)geq[0]);
            }
        } else if (bb) {
            stp<S, OPP[i]>(row, v, co, (R)(feq[i] - rest_f(v, OPP[i])));
            stp<S, 9 + OPP[i]>(row, v, co, (R)geq[i]);
        } else {
            stp<S, i>(row, v, co, (R)(feq[i] - rest_f(v, i)));
            stp<S, 9 + i>(row, v, co, (R)geq[i]);
        }
    });
}

// ------------------------------------------------------------------ read-back

// Moments of S_n at the nodes first .. first+count-1 (host order): optional
// compact FP64 fields (phi, rho, ux, uy planes of count values) and FP64
// partial records of sums over fluid nodes (sum rho, sum phi, kinetic energy,
// max |u|, count, and sum (1+phi)/2 for x in [x_lo, x_hi)).
template <int S>
__global__ __launch_bounds__(256) void moments_kernel(View v, int parity, int64_t first,
                                                      int64_t count,
                                                      double* __restrict__ fields,
                                                      double* __restrict__ partials,
                                                      int32_t x_lo, int32_t x_hi) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t id = first + k;
    double a[6] = {0, 0, 0, 0, 0, 0};
    if (k < count) {
        const int x = (int)(id % v.nx), y = (int)(id / v.nx);
        double ph = 0, rho = 0, ux = 0, uy = 0;
        double f[9], g[9];
        if (pull_node_abs<S>(v, parity, x, y, f, g)) {
            double jx = 0, jy = 0;
            for (int i = 0; i < 9; ++i) {
                rho += f[i];
                ph += g[i];
                jx += EX[i] * f[i];
                jy += EY[i] * f[i];
            }
            ux = jx / rho;
            uy = jy / rho;
            const double u2 = ux * ux + uy * uy;
            a[0] = rho;
            a[1] = ph;
            a[2] = 0.5 * rho * u2;
            a[3] = sqrt(u2);
            a[4] = 1.0;
            if (x >= x_lo && x < x_hi) a[5] = 0.5 * (1.0 + ph);
        }
        if (fields) {
            fields[k] = ph;
            fields[count + k] = rho;
            fields[2 * count + k] = ux;
            fields[3 * count + k] = uy;
        }
    }
    if (partials) {
        __shared__ double red[4][6];
#pragma unroll
        for (int k = 0; k < 6; ++k) {
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) {
                const double b = __shfl_xor(a[k], off, 64);
                a[k] = k == 3 ? ((b > a[k] || b != b) ? b : a[k]) : a[k] + b;
            }
        }
        const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
        if (lane == 0)
            for (int k = 0; k < 6; ++k) red[wv][k] = a[k];
        __syncthreads();
        if (threadIdx.x == 0) {
            double* o = partials + (int64_t)blockIdx.x * kPartials;
            for (int k = 0; k < 6; ++k) o[k] = 0;
            for (int w = 0; w < 4; ++w) {
                for (int k = 0; k < 6; ++k)
                    if (k == 3)
                        o[3] = (red[w][3] > o[3] || red[w][3] != red[w][3]) ? red[w][3] : o[3];
                    else
                        o[k] += red[w][k];
            }
        }
    }
}

// One population plane of S_n (pulled) as compact FP64 nx*ny; zero at solid nodes.
template <int S>
__global__ __launch_bounds__(256) void read_plane_kernel(View v, int parity, int plane,
                                                         double* __restrict__ out) {
    const int64_t n = (int64_t)v.nx * v.ny;
    const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= n) return;
    const int x = (int)(id % v.nx), y = (int)(id / v.nx);
    double f[9], g[9];
    if (!pull_node_abs<S>(v, parity, x, y, f, g)) {
        out[id] = 0.0;
        return;
    }
    double val = 0.0;
    for (int i = 0; i < 9; ++i) val = (i == plane) ? f[i] : ((i == plane - 9) ? g[i] : val);
    out[id] = val;
}

// phi = 0 crossings on the +x and +y links of every fluid node whose far end
// is fluid and of opposite sign (Sec. IV); compacted with an atomic counter.
template <int S>
__global__ __launch_bounds__(256) void crossings_kernel(View v, int parity,
                                                        Crossing* __restrict__ pts,
                                                        int64_t capacity,
                                                        unsigned long long* __restrict__ counter) {
    const int64_t n = (int64_t)v.nx * v.ny;
    const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= n) return;
    const int x = (int)(id % v.nx), y = (int)(id / v.nx);
    const int nx = v.nx, ny = v.ny;
    auto phi_at = [&](int xx, int yy, bool& fluid) -> double {
        double f[9], g[9];
        fluid = pull_node_abs<S>(v, parity, xx, yy, f, g);
        if (!fluid) return 0.0;
        double s = 0;
        for (int i = 0; i < 9; ++i) s += g[i];
        return s;
    };
    bool fa;
    const double a = phi_at(x, y, fa);
    if (!fa) return;
    for (int axis = 0; axis < 2; ++axis) {
        const int x2 = axis == 0 ? (x == nx - 1 ? 0 : x + 1) : x;
        const int y2 = axis == 0 ? y : (y == ny - 1 ? 0 : y + 1);
        bool fb;
        const double b = phi_at(x2, y2, fb);
        if (!fb) continue;
        if ((a > 0 && b < 0) || (a < 0 && b > 0)) {
            const unsigned long long k = atomicAdd(counter, 1ull);
            if ((int64_t)k < capacity) {
                Crossing c;
                c.key = ((uint64_t)id << 2) | ((uint64_t)axis << 1) | (a > 0 ? 1u : 0u);
                c.t = a / (a - b);
                pts[k] = c;
            }
        }
    }
}

// Streaming copies used as a reference for the device's HBM read + write rate.
// Variant 0: one 16-byte element per thread and iteration, plain loads and
// stores; 1: four elements in flight per thread, plain loads, nontemporal
// stores (as the sweep stores); 2: four elements, nontemporal loads and stores.
typedef float f32x4 __attribute__((ext_vector_type(4)));
template <int V>
__global__ __launch_bounds__(256) void stream_copy_kernel(const f32x4* __restrict__ src,
                                                          f32x4* __restrict__ dst, size_t n) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if constexpr (V > 0) {
        for (; i + 3 * stride < n; i += 4 * stride) {
            f32x4 v[4];
#pragma unroll
            for (int u = 0; u < 4; ++u)
                v[u] = V == 2 ? __builtin_nontemporal_load(src + i + u * stride) : src[i + u * stride];
#pragma unroll
            for (int u = 0; u < 4; ++u) __builtin_nontemporal_store(v[u], dst + i + u * stride);
        }
    }
    for (; i < n; i += stride) dst[i] = src[i];
}

hipError_t launch_stream_copy(const void* src, void* dst, size_t bytes, int blocks, int variant,
                              hipStream_t stream) {
    const f32x4* a = reinterpret_cast<const f32x4*>(src);
    f32x4* b = reinterpret_cast<f32x4*>(dst);
    const size_t n = bytes / sizeof(f32x4);
    if (variant == 0) hipLaunchKernelGGL(stream_copy_kernel<0>, dim3(blocks), dim3(256), 0, stream, a, b, n);
    else if (variant == 1) hipLaunchKernelGGL(stream_copy_kernel<1>, dim3(blocks), dim3(256), 0, stream, a, b, n);
    else hipLaunchKernelGGL(stream_copy_kernel<2>, dim3(blocks), dim3(256), 0, stream, a, b, n);
    return hipGetLastError();
}

__global__ void fill_kernel(uint8_t* __restrict__ p, uint8_t value, size_t bytes) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t k = i; k < bytes; k += stride) p[k] = value;
}

hipError_t launch_finalize(const Tile*, const int32_t* member_first, int n_members,
                           int n_records_single, const double* partials, double* diag_out,
                           int32_t* flag, hipStream_t stream) {
    hipLaunchKernelGGL(finalize_kernel, dim3(n_members), dim3(256), 0, stream, member_first,
                       n_records_single, partials, diag_out, flag);
    return hipGetLastError();
}

static inline unsigned blocks_for(int64_t n) { return (unsigned)((n + 255) / 256); }

#define LB_DISPATCH_STORAGE(st, KERNEL, grid, ...)                                          \
    switch (st) {                                                                           \
        case ST_F64: hipLaunchKernelGGL(KERNEL<ST_F64>, grid, dim3(256), 0, __VA_ARGS__); break; \
        case ST_F32: hipLaunchKernelGGL(KERNEL<ST_F32>, grid, dim3(256), 0, __VA_ARGS__); break; \
        case ST_F16S: hipLaunchKernelGGL(KERNEL<ST_F16S>, grid, dim3(256), 0, __VA_ARGS__); break; \
        case ST_BF16S: hipLaunchKernelGGL(KERNEL<ST_BF16S>, grid, dim3(256), 0, __VA_ARGS__); break; \
        case ST_F64C: hipLaunchKernelGGL(KERNEL<ST_F64C>, grid, dim3(256), 0, __VA_ARGS__); break; \
        case ST_F32C: hipLaunchKernelGGL(KERNEL<ST_F32C>, grid, dim3(256), 0, __VA_ARGS__); break; \
        default: return hipErrorInvalidValue;                                               \
    }

hipError_t launch_init_state(const View& v, const double* phi0, const double* rho0,
                             const double* ux0, const double* uy0, hipStream_t stream) {
    const dim3 grid(blocks_for((int64_t)v.nx * v.ny));
    LB_DISPATCH_STORAGE(v.storage, init_kernel, grid, stream, v, phi0, rho0, ux0, uy0);
    return hipGetLastError();
}

hipError_t launch_moments(const View& v, int parity, int64_t first, int64_t count,
                          double* fields, double* partials, int n_records, int32_t x_lo,
                          int32_t x_hi, hipStream_t stream) {
    if (first < 0 || count <= 0 || first + count > (int64_t)v.nx * v.ny) return hipErrorInvalidValue;
    const dim3 grid(blocks_for(count));
    if (partials && (int64_t)grid.x > n_records) return hipErrorInvalidValue;
    LB_DISPATCH_STORAGE(v.storage, moments_kernel, grid, stream, v, parity, first, count, fields,
                        partials, x_lo, x_hi);
    return hipGetLastError();
}

hipError_t launch_read_plane(const View& v, int parity, int plane, double* out,
                             hipStream_t stream) {
    const dim3 grid(blocks_for((int64_t)v.nx * v.ny));
    LB_DISPATCH_STORAGE(v.storage, read_plane_kernel, grid, stream, v, parity, plane, out);
    return hipGetLastError();
}

hipError_t launch_crossings(const View& v, int parity, void* points, int64_t capacity,
                            unsigned long long* counter, hipStream_t stream) {
    const dim3 grid(blocks_for((int64_t)v.nx * v.ny));
    Crossing* pts = reinterpret_cast<Crossing*>(points);
    LB_DISPATCH_STORAGE(v.storage, crossings_kernel, grid, stream, v, parity, pts, capacity,
                        counter);
    return hipGetLastError();
}

hipError_t launch_fill(void* dst, uint8_t value, size_t bytes, hipStream_t stream) {
    if (bytes == 0) return hipSuccess;
    const size_t blocks = (bytes + 255) / 256;
    const unsigned g = (unsigned)(blocks < 65536 ? blocks : 65536);
    hipLaunchKernelGGL(fill_kernel, dim3(g), dim3(256), 0, stream,
                       reinterpret_cast<uint8_t*>(dst), value, bytes);
    return hipGetLastError();
}

#endif  // LB_SWEEP_UNIT

}  // namespace lbm
