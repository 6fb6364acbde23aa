// Learned preconditioner: a 4-layer 3x3x3 convolution network (channels
// 2 -> 16 -> 16 -> 16 -> 1, ReLU after the first three) applied inside
// flexible CG, and its training kernels.
//
// Convolutions are implicit GEMMs on the matrix cores with
// v_mfma_f32_16x16x32_bf16 (BF16 operands, FP32 accumulation). A block owns a
// 1 x 4 x 64 tile of output cells; each of its four waves computes one 64-cell
// row as four 16-cell tiles. Activations are stored channels-last in BF16
// (32 bytes per cell for 16 channels).
//
// 16-channel inputs: the z taps are applied on the output side. For a pair of
// (dx, dy) tap groups, one 16-cell x 32-channel slab of the input (16 channels
// of each group, unshifted, from an LDS tile with a one-cell halo) is the B
// operand of three products, one per z offset dz, Q_dz = W_dz x; the output is
// y[z] = Q_-1[z-1] + Q_0[z] + Q_+1[z+1], the z neighbours taken across lanes.
// Each input slab is read from LDS once per pair instead of once per tap. A
// fifth tile holds the two cells just beyond the row ends. The first layer's
// two input channels are packed as (tap, channel) pairs into K = 64 (54 used).
//
// Backward: the input gradient is the forward convolution of the output
// gradient with the taps mirrored and the channel roles swapped, followed by
// the ReLU mask of the layer below; the weight gradient is a GEMM over cells,
// D[ci][co] += x[cell + off][ci] * dy[cell][co], with per-block partials
// summed in a fixed order by a second kernel. Adam updates FP32 master
// weights and rebuilds the BF16 operand layouts.
#include "nn.hpp"
#include "launch.hpp"

#include <atomic>
#include <cmath>
#include <cstring>
#include <string>
#include <type_traits>
#include <vector>

namespace mffv {
namespace {

typedef short v4s __attribute__((ext_vector_type(4)));
typedef short v8s __attribute__((ext_vector_type(8)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef float v4f __attribute__((ext_vector_type(4)));

// D += A B on a 16 x 16 x 32 BF16 tile. Lane l holds A row l % 16 and B
// column l % 16, each with the 8 K values of slot l / 16; it receives D rows
// 4 (l / 16) .. 4 (l / 16) + 3 of column l % 16.
__device__ __forceinline__ v4f mfma32(const v8s& a, const v8s& b, const v4f& c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(v8bf, a), __builtin_bit_cast(v8bf, b), c,
                                                   0, 0, 0);
}

constexpr int TZ = 64, TY = 4;                  // output tile: 1 x TY x TZ cells
constexpr int HX = 3, HY = TY + 2, HZ = TZ + 2;  // input tile with a one-cell halo
constexpr int HCELLS = HX * HY * HZ;

// parameter offsets of the FP32 master vector: per layer W[27][cin][cout], b[cout]
constexpr int kCin[4] = {2, 16, 16, 16};
constexpr int kCout[4] = {16, 16, 16, 1};
constexpr int offW(int l) {
    int o = 0;
    for (int i = 0; i < l; ++i) o += 27 * kCin[i] * kCout[i] + kCout[i];
    return o;
}
constexpr int offB(int l) { return offW(l) + 27 * kCin[l] * kCout[l]; }
constexpr int kNParams = offW(4);
static_assert(kNParams == 15169, "parameter count");

// BF16 A-operand layouts of the weights (v8s per lane, 64 lanes per operand):
// forward and input-gradient (mirrored taps, channel roles swapped).
//  2-channel input (layer 1, input gradient of layer 4): 2 operands, K = 64
//    (tap, channel) pairs, k = 2 tap + channel.
//  16-channel input, 16 outputs: 4 pairs of (dx, dy) groups x 3 dz operands
//    (pair P: groups 2P and 2P+1 in K halves), then group 8 with its z taps
//    in K: [W_-1 | W_0] and [W_+1 | 0] (a 15th, zero operand keeps the stride).
//  16-channel input, 1 output (layer 4): 5 pair operands with rows = dz + 1.
constexpr int kPairs = 5;
constexpr int kWf1 = 0;
constexpr int kWf2 = kWf1 + 2 * 64;
constexpr int kWf3 = kWf2 + 3 * kPairs * 64;
constexpr int kWf4 = kWf3 + 3 * kPairs * 64;
constexpr int kWb4 = kWf4 + kPairs * 64;
constexpr int kWb3 = kWb4 + 2 * 64;
constexpr int kWb2 = kWb3 + 3 * kPairs * 64;
constexpr int kWTotal = kWb2 + 3 * kPairs * 64;  // in v8s units

typedef float v2f __attribute__((ext_vector_type(2)));
typedef __bf16 v2bf __attribute__((ext_vector_type(2)));
// FP32 -> BF16, round to nearest even (v_cvt_pk_bf16_f32: two values at once).
__device__ __forceinline__ uint32_t pack_bf2(float lo, float hi) {
    return __builtin_bit_cast(uint32_t, __builtin_convertvector((v2f){lo, hi}, v2bf));
}
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint16_t f2bf(float f) { return (uint16_t)pack_bf2(f, 0.f); }
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

struct Tile {
    int i, j0, k0;
};
__device__ __forceinline__ Tile tile_of(int t, int ntj, int ntk) {
    Tile T;
    T.k0 = (t % ntk) * TZ;
    T.j0 = ((t / ntk) % ntj) * TY;
    T.i = t / (ntk * ntj);
    return T;
}
__device__ __forceinline__ int hcell(int hx, int hy, int hz) { return (hx * HY + hy) * HZ + hz; }

// Load the haloed input tile of a channels-last BF16 tensor with C channels.
template <int C>
__device__ __forceinline__ void load_halo(const uint16_t* __restrict__ in, const Geom& g, Tile T,
                                          uint16_t* lds) {
    if (C == 16) {
        for (int c = threadIdx.x; c < HCELLS * 2; c += kThreads) {
            const int cell = c >> 1, half = c & 1;
            const int hz = cell % HZ, hy = (cell / HZ) % HY, hx = cell / (HZ * HY);
            const int i = T.i - 1 + hx, j = T.j0 - 1 + hy, k = T.k0 - 1 + hz;
            uint4 v = make_uint4(0, 0, 0, 0);
            if (i >= 0 && i < g.nx && j >= 0 && j < g.ny && k >= 0 && k < g.nz) {
                const int64_t l = ((int64_t)i * g.ny + j) * g.nz + k;
                v = *reinterpret_cast<const uint4*>(in + l * 16 + half * 8);
            }
            *reinterpret_cast<uint4*>(lds + cell * 16 + half * 8) = v;
        }
    } else {
        for (int cell = threadIdx.x; cell < HCELLS; cell += kThreads) {
            const int hz = cell % HZ, hy = (cell / HZ) % HY, hx = cell / (HZ * HY);
            const int i = T.i - 1 + hx, j = T.j0 - 1 + hy, k = T.k0 - 1 + hz;
            uint32_t v = 0;
            if (i >= 0 && i < g.nx && j >= 0 && j < g.ny && k >= 0 && k < g.nz) {
                const int64_t l = ((int64_t)i * g.ny + j) * g.nz + k;
                v = *reinterpret_cast<const uint32_t*>(in + l * 2);
            }
            *reinterpret_cast<uint32_t*>(lds + cell * 2) = v;
        }
    }
}

// Forward and input-gradient convolutions march along x: a block owns a
// column of TY x TZ output cells and a run of consecutive x planes, so every
// input plane is read from memory once per run instead of three times. The
// haloed input planes go from memory straight into a ring of kRingSlots LDS
// slots (global_load_lds, no registers in between); plane p is requested at
// the start of step p - kAhead, so while the matrix cores work on plane i
// (slots of planes i-1, i, i+1) the planes up to i + kAhead are in flight.
// Four slots (plane p is requested one step before it is needed) keep a
// block's LDS at 52 KiB, so that three blocks (three waves per SIMD) fit a
// CU: measured faster than six slots at two blocks per CU.
constexpr int kRingSlots = 4;
constexpr int kAhead = kRingSlots - 2;  // the slot of plane p + kAhead was last read at step p - 1
constexpr int PCELLS = HY * HZ;         // cells of one haloed plane

// In LDS the two 16-byte channel halves of a 16-channel cell are stored in the
// order h ^ ((cell >> 3) & 1): the 16 lanes that read half h of 16 consecutive
// cells then cover all 64 banks once instead of half of them twice.
__device__ __forceinline__ int half_pos(int cell, int h) { return cell * 16 + ((h ^ (cell >> 3)) & 1) * 8; }

typedef __attribute__((address_space(3))) uint16_t lds16;
typedef __attribute__((address_space(3))) void lds_void;

// Source of the halo cells outside the grid and of the planes past a block's
// run: 16 zero bytes.
__device__ __attribute__((aligned(16))) uint32_t g_zero16[4];
// Buffer resource word 3 (CDNA: untyped 32-bit data format, raw addressing)
// and the cache-policy bit of a nontemporal access.
constexpr int kBufWord3 = 0x00020000;
constexpr int kNonTemporal = 2;
// Destination of the stores of lanes without an output cell: every store
// instruction is issued by every wave that has a row, so the number of memory
// operations a wave has in flight is known at each step.
__device__ __attribute__((aligned(16))) uint32_t g_trash[64 * 4];

// A plane is moved in 16-byte units (16 channels: cell, stored half) or
// 4-byte units (2 channels: cell), 64 per wave instruction; wave w issues the
// instructions 4 u + w. A slot holds a whole number of instructions' units
// (the lanes past the plane's last unit write zeros into the padding).
template <int C>
constexpr int plane_units() { return C == 16 ? 2 * PCELLS : PCELLS; }
template <int C>
constexpr int plane_groups() { return (plane_units<C>() + 63) / 64; }
template <int C>
constexpr int slot_u16() { return plane_groups<C>() * 64 * (C == 16 ? 8 : 2); }  // slot stride, uint16 units
template <int C>
__device__ __forceinline__ int dma_per_plane(int w) { return (plane_groups<C>() - w + 3) / 4; }

// Per lane and instruction u: where in an x plane of the input (uint16 units)
// the unit this lane moves comes from, or -1 for zeros (halo cells outside the
// grid, padding). Lane data lands at slot + 64 (4 u + w) size + lane size, so
// the lane of unit c reads the global half that belongs there.
template <int C>
__device__ __forceinline__ void dma_offsets(const Geom& g, int j0, int k0, int doff[4]) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int c = (4 * u + w) * 64 + lane;
        int off = -1;
        if (c < plane_units<C>()) {
            const int cell = C == 16 ? c >> 1 : c;
            const int j = j0 - 1 + cell / HZ, k = k0 - 1 + cell % HZ;
            if (j >= 0 && j < g.ny && k >= 0 && k < g.nz)
                off = C == 16 ? (j * g.nz + k) * 16 + ((c & 1) ^ ((cell >> 3) & 1)) * 8 : (j * g.nz + k) * 2;
        }
        doff[u] = off;
    }
}

// One LDS DMA instruction: every lane moves BYTES from src to the wave's
// destination + lane * BYTES (M0 holds the destination; the nop separates
// the M0 write from its use). Written as asm,
// with no output register: the compiler then does not know of an LDS write
// in flight and keeps exact LDS wait counts for the reads of the other slots
// (with the builtin it waits for every LDS read at once). The march waits for
// these requests itself (wait_vmcnt, before the barrier that publishes a slot).
template <int BYTES>
__device__ __forceinline__ void lds_dma(const void* src, lds16* dst) {
    const uint32_t m0 = __builtin_amdgcn_readfirstlane((uint32_t)(uintptr_t)dst);
    if constexpr (BYTES == 16)
        asm volatile("s_nop 0\n\tglobal_load_lds_dwordx4 %0, off" ::"v"(src), "{m0}"(m0) : "memory");
    else
        asm volatile("s_nop 0\n\tglobal_load_lds_dword %0, off" ::"v"(src), "{m0}"(m0) : "memory");
}

// Request haloed plane i (zeros if the block does not need it or it lies
// outside the grid) into an LDS slot.
template <int C>
__device__ __forceinline__ void dma_plane(const uint16_t* __restrict__ in, const Geom& g, int i, bool need,
                                          const int doff[4], lds16* __restrict__ slot) {
    const int w = threadIdx.x >> 6;
    const bool iin = need && i >= 0 && i < g.nx;
    const uint16_t* base = in + (int64_t)i * g.ny * g.nz * C;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int grp = 4 * u + w;
        if (grp >= plane_groups<C>()) break;
        const void* src = iin && doff[u] >= 0 ? (const void*)(base + doff[u]) : (const void*)g_zero16;
        lds_dma<C == 16 ? 16 : 4>(src, slot + grp * 64 * (C == 16 ? 8 : 2));
    }
}

// s_waitcnt vmcnt(n): wait until at most n vector memory operations of this
// wave are in flight (they complete in issue order). n is wave-uniform.
#define MFFV_VMCNT(n) ((n & 15) | ((n >> 4) << 14) | (7 << 4) | (15 << 8))
__device__ __forceinline__ void wait_vmcnt(int n) {
    switch (n < 0 ? 0 : n) {
#define MFFV_WAIT_CASE(n) case n: __builtin_amdgcn_s_waitcnt(MFFV_VMCNT(n)); break;
        MFFV_WAIT_CASE(0) MFFV_WAIT_CASE(1) MFFV_WAIT_CASE(2) MFFV_WAIT_CASE(3) MFFV_WAIT_CASE(4)
        MFFV_WAIT_CASE(5) MFFV_WAIT_CASE(6) MFFV_WAIT_CASE(7) MFFV_WAIT_CASE(8) MFFV_WAIT_CASE(9)
        MFFV_WAIT_CASE(10) MFFV_WAIT_CASE(11) MFFV_WAIT_CASE(12) MFFV_WAIT_CASE(13) MFFV_WAIT_CASE(14)
        MFFV_WAIT_CASE(15) MFFV_WAIT_CASE(16) MFFV_WAIT_CASE(17) MFFV_WAIT_CASE(18) MFFV_WAIT_CASE(19)
        MFFV_WAIT_CASE(20) MFFV_WAIT_CASE(21) MFFV_WAIT_CASE(22) MFFV_WAIT_CASE(23)
#undef MFFV_WAIT_CASE
        default: __builtin_amdgcn_s_waitcnt(MFFV_VMCNT(24)); break;
    }
}
#undef MFFV_VMCNT

// Workgroup barrier without a memory fence: the LDS data the waves exchange
// arrives by global_load_lds, whose completion each wave waits for itself
// (wait_vmcnt) before the barrier. The asm's memory clobber keeps the compiler
// from moving memory accesses across it.
__device__ __forceinline__ void ring_barrier() { asm volatile("s_barrier" ::: "memory"); }

// Row rotations have a source for every lane, so bound_ctrl changes nothing;
// set, it lets the compiler fold the move into the add that uses it.
__device__ __forceinline__ float dpp_ror1(float v) {   // lane i of each 16-lane row gets lane i - 1 (mod 16)
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x121, 0xf, 0xf, true));
}
__device__ __forceinline__ float dpp_rol1(float v) {   // lane i of each 16-lane row gets lane i + 1 (mod 16)
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x12f, 0xf, 0xf, true));
}

// Where lane (q, n) reads the B operand of (dx, dy) group pair P: group
// 2P + (q >> 1) (the second group of pair 4 is empty: it reads the first
// group's cells, which meet zero weights), channel half q & 1. dx picks the
// plane; off is the offset in the plane (uint16 units) of tile 0 (cell n of
// the row), halo the offset for the halo tile (column 15: the cell before the
// row, the other columns: the cell after it). Tile t adds 256 t: 16 cells
// further along z, the same swizzle (16 t does not change cell >> 3).
struct SlabAt {
    int dx, off, halo;
};
__device__ __forceinline__ SlabAt slab_at(int P) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int n = lane & 15, q = lane >> 4;
    const int g = min(2 * P + (q >> 1), 8);
    const int row = (w + g % 3) * HZ;
    const int hz = n == 15 ? 0 : HZ - 1;
    return SlabAt{g / 3, half_pos(row + n + 1, q & 1), half_pos(row + hz, q & 1)};
}

// base: the ring; so[d]: offset of the slot of plane i - 1 + d (uint16 units).
__device__ __forceinline__ v8s slab(const lds16* base, const int so[3], const SlabAt& a, int t) {
    typedef __attribute__((address_space(3))) const v8s lds_v8s;
    return *reinterpret_cast<lds_v8s*>(base + so[a.dx] + (t < 4 ? a.off + 256 * t : a.halo));
}

// One wave's 64-cell output row of a 16 -> 16 convolution, tile by tile.
// Group pairs 0-3 ((dx, dy) groups 0-7) take the z taps on the output side:
// Q_dz = W_dz x (dz = -1, 0, 1), y[z] = Q_-1[z-1] + Q_0[z] + Q_+1[z+1] across
// the 16-lane rows of cells. Group 8 takes them on the input side, in two
// products into Q_0: [W_-1 | W_0] [x(z-1); x(z)] and [W_+1 | 0] [x(z+1); -]
// (14 products a tile instead of 15 with a half-empty fifth pair, and no halo
// products for group 8). Tile t - 1 is finished, and handed to epi(t - 1, y)
// (lane (q, n): output channels 4q..4q+3 of cell n of that tile), once tile
// t's Q_+1 exists; its vector work is independent of tile t + 1's products,
// so the two overlap. The halo tile holds the cell before the row (column
// 15, dz = -1) and the cell after it (the other columns, dz = +1) for pairs
// 0-3; hb / ha: those cells lie in the grid (outside it they are zeros and
// their products are skipped). wr: 14 operands, 3 P + dz + 1 for P < 4, then
// group 8's two.
template <class Epi>
__device__ __forceinline__ void conv_row16(const lds16* base, const int so[3], const v8s* wr, bool hb, bool ha,
                                           Epi&& epi) {
    typedef __attribute__((address_space(3))) const v8s lds_v8s;
    constexpr int kOut = kPairs - 1;  // pairs with the z taps on the output side
    constexpr int kPer = kOut + 2;    // slab reads per tile
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int n = lane & 15, q = lane >> 4;
    int ad[kPer], ah[kOut];
#pragma unroll
    for (int P = 0; P < kOut; ++P) {
        const SlabAt at = slab_at(P);
        ad[P] = so[at.dx] + at.off;
        ah[P] = so[at.dx] + at.halo;
    }
    {   // group 8 (dx = +1, dy = +1): cell n - 1 | n, then cell n + 1, of tile 0
        const int row = (w + 2) * HZ, h = q & 1;
        ad[kOut] = so[2] + half_pos(row + n + (q >> 1), h);
        ad[kOut + 1] = so[2] + half_pos(row + n + 2, h);
    }
    auto rd = [&](int off) { return *reinterpret_cast<lds_v8s*>(base + off); };
    // the row's 24 slabs in the order they are used (s = 6 t + e), read two
    // ahead of their products through a ring of three
    auto slab_off = [&](int s) { return ad[s % kPer] + 256 * (s / kPer); };  // 16 cells further per tile
    v8s ring[3];
    ring[0] = rd(slab_off(0));
    ring[1] = rd(slab_off(1));
    v4f H0 = v4f{0.f, 0.f, 0.f, 0.f}, H1 = H0;
    if (hb || ha) {
        v8s bh[kOut];
#pragma unroll
        for (int P = 0; P < kOut; ++P) bh[P] = rd(ah[P]);
        // (straight-line code per case)
        if (hb && ha) {
#pragma unroll
            for (int P = 0; P < kOut; ++P) {
                H0 = mfma32(wr[3 * P + 0], bh[P], H0);
                H1 = mfma32(wr[3 * P + 2], bh[P], H1);
            }
        } else if (hb) {
#pragma unroll
            for (int P = 0; P < kOut; ++P) H0 = mfma32(wr[3 * P + 0], bh[P], H0);
        } else {
#pragma unroll
            for (int P = 0; P < kOut; ++P) H1 = mfma32(wr[3 * P + 2], bh[P], H1);
        }
    }
    v4f L = H0, A, R;  // previous tile: its dz = -1 products, Q_0 + left part, dz = +1 products
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        v4f Q0 = v4f{0.f, 0.f, 0.f, 0.f}, Q1 = Q0, Q2 = Q0;
#pragma unroll
        for (int e = 0; e < kPer; ++e) {
            const int sidx = kPer * t + e;
            if (sidx + 2 < 4 * kPer) ring[(sidx + 2) % 3] = rd(slab_off(sidx + 2));
            const v8s b = ring[sidx % 3];
            if (e < kOut) {
                Q0 = mfma32(wr[3 * e + 0], b, Q0);
                Q1 = mfma32(wr[3 * e + 1], b, Q1);
                Q2 = mfma32(wr[3 * e + 2], b, Q2);
            } else {
                Q1 = mfma32(wr[3 * kOut + e - kOut], b, Q1);
            }
            if (sidx + 2 < 4 * kPer) __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
            if (e < kOut) __builtin_amdgcn_sched_group_barrier(0x008, 3, 0);
            else __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
        }
        if (t > 0) {
            v4f y;
#pragma unroll
            for (int v = 0; v < 4; ++v) y[v] = A[v] + dpp_rol1(n == 0 ? Q2[v] : R[v]);
            epi(t - 1, y);
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) A[v] = Q1[v] + dpp_ror1(n == 15 ? L[v] : Q0[v]);
        R = Q2;
        L = Q0;
    }
    v4f y;
#pragma unroll
    for (int v = 0; v < 4; ++v) y[v] = A[v] + dpp_rol1(n == 0 ? H1[v] : R[v]);
    epi(3, y);
}

// Per-lane offsets (uint16 units from the slot of plane i - 1) of the eight
// (tap, channel-pair) reads of a 2 -> 16 convolution: tap = 16 s + 4 q + j for
// K slot s, lane group q, j = 0..3 (taps past 26 read tap 26's cell, which
// meets zero weights); plane dx lies dx slots further (the ring's first two
// slots are mirrored past its end). Computed once per kernel: decoding the
// taps per lane in the loop costs more than the matrix work.
constexpr int SLOT2 = slot_u16<2>();
__device__ __forceinline__ void tap_offsets2(int toff[8]) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int n = lane & 15, q = lane >> 4;
#pragma unroll
    for (int s2 = 0; s2 < 2; ++s2)
#pragma unroll
        for (int jj = 0; jj < 4; ++jj) {
            const int tap = min(16 * s2 + 4 * q + jj, 26);
            const int dx = tap / 9, dy = (tap / 3) % 3, dz = tap % 3;
            toff[4 * s2 + jj] = dx * SLOT2 + ((w + dy) * HZ + n + dz) * 2;
        }
}

// One wave's 64-cell output row of a 2 -> 16 convolution: K = 64 (tap,
// channel) pairs in two products per tile, k = 32 s + 8 q + v, tap = k / 2,
// channel = k % 2; each lane gathers the 4-byte cells of its four taps.
__device__ __forceinline__ void conv_row2(const lds16* base, const int toff[8], const v8s* wr, v4f y[4]) {
#pragma unroll
    for (int t = 0; t < 4; ++t) y[t] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int s = 0; s < 2; ++s) {
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            uint32_t c[4];
#pragma unroll
            for (int j = 0; j < 4; ++j)
                c[j] = *reinterpret_cast<__attribute__((address_space(3))) const uint32_t*>(base + toff[4 * s + j] + 32 * t);
            y[t] = mfma32(wr[s], __builtin_bit_cast(v8s, make_uint4(c[0], c[1], c[2], c[3])), y[t]);
        }
    }
}

// The last layer (16 -> 1 channel) of one wave's 64-cell row: the A rows are
// the three z offsets (row dz + 1), so one product per pair and tile gives
// Q_dz for every dz; the output is Q_-1[z-1] + Q_0[z] + Q_+1[z+1]. Returns, on
// lanes 0..15, the outputs of cells n, n+16, n+32, n+48 of the row.
__device__ __forceinline__ void conv_last_row(const lds16* base, const int so[3], const v8s* wz, float y[4]) {
    const int n = threadIdx.x & 15;
    v4f Q[5];
#pragma unroll
    for (int t = 0; t < 5; ++t) Q[t] = v4f{0.f, 0.f, 0.f, 0.f};
    v8s B[2][5];
    {
        const SlabAt at = slab_at(0);
#pragma unroll
        for (int t = 0; t < 5; ++t) B[0][t] = slab(base, so, at, t);
    }
#pragma unroll
    for (int P = 0; P < kPairs; ++P) {
        __builtin_amdgcn_sched_barrier(0);
        const int cur = P & 1;
        if (P + 1 < kPairs) {
            const SlabAt at = slab_at(P + 1);
#pragma unroll
            for (int t = 0; t < 5; ++t) B[cur ^ 1][t] = slab(base, so, at, t);
        }
#pragma unroll
        for (int t = 0; t < 5; ++t) Q[t] = mfma32(wz[P], B[cur][t], Q[t]);
        if (P + 1 < kPairs) __builtin_amdgcn_sched_group_barrier(0x100, 5, 0);
        __builtin_amdgcn_sched_group_barrier(0x008, 5, 0);
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const float lsel = n == 15 ? (t > 0 ? Q[t - 1][0] : Q[4][0]) : Q[t][0];
        const float rsel = n == 0 ? (t < 3 ? Q[t + 1][2] : Q[4][2]) : Q[t][2];
        y[t] = Q[t][1] + dpp_ror1(lsel) + dpp_rol1(rsel);
    }
}

enum ConvOut {
    kHiddenRelu = 0,  // + bias, ReLU, BF16 16 channels
    kGradMasked = 1,  // input gradient: x (h_below > 0), BF16 16 channels
    kFinal = 2,       // + bias, channel 0 only, FP32 (training output)
    kPrecond = 3,     // + bias, z = dinv r + s sqrt(dinv) y on unknown cells, 0 on Dirichlet
};

struct ConvArgs {
    const uint16_t* in;
    const v8s* W;
    const float* bias;      // kHiddenRelu, kFinal, kPrecond
    uint16_t* out16;        // kHiddenRelu, kGradMasked
    const uint16_t* below;  // kGradMasked: activation of the layer below (ReLU mask)
    float* out32;           // kFinal, kPrecond
    const float* r;         // kPrecond
    const float* dinv;
    const uint8_t* dmask;
    const float* sscale;    // kPrecond: device scalar s
    const float* r1;        // kPrecond with the Jacobi sweeps: the residual after the first sweep
    float omega;            //   and the sweeps' weight
    int relu;               // 1: ReLU after the hidden layers, 0: identity
    int ntk;                // column tiles along z
    int ncols;              // column tiles in total (y tiles x z tiles)
    int run;                // x planes per block
    const int* done;        // optional: the CG loop's done flag (return at once once set)
    const float* in_scale;  // first layer, optional: device scalar multiplying its products (the
                            //   network input's 1/s, a power of two, when the input is unscaled)
};


// Slot after slot x of the ring.
__device__ __forceinline__ int ring_next(int x, int d) { return x + d >= kRingSlots ? x + d - kRingSlots : x + d; }

// One step of the x march: request plane i + kAhead, then compute output plane
// i from the slots of planes i-1, i, i+1 (sl: slot of plane i-1) and store it.
// The LDS reads go through rd and the request through rq, both restrict (they
// address different slots): the compiler then does not make the reads wait
// for the request.
// The epilogue's own per-cell operands of one output row (last layer in
// flexible CG: r, dinv, dmask and the swept residual; input gradient: the
// activation of the layer below, for its ReLU mask).
struct EpiIn {
    float r[4], d[4], r1[4];
    uint8_t m[4];
    uint2 b[4];
};

// Load them for plane i, by every lane from a clamped (always valid) address
// and without branches. The march loads them one step ahead, after that
// step's plane request: since memory operations complete in issue order,
// waiting for them then waits only for requests at least a step old.
template <int MODE>
__device__ __forceinline__ void epi_load(const Geom& g, const ConvArgs& a, int i, int j0, int k0, EpiIn& e) {
    if (MODE != kPrecond && MODE != kGradMasked) return;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int m = lane & 15, rg = lane >> 4;
    const int64_t rowc = ((int64_t)min(i, g.nx - 1) * g.ny + min(j0 + w, g.ny - 1)) * g.nz;
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
        const int64_t l = rowc + min(k0 + mt * 16 + m, g.nz - 1);
        if (MODE == kPrecond) {
            e.r[mt] = a.r[l];
            e.d[mt] = a.dinv[l];
            e.m[mt] = a.dmask[l];
            e.r1[mt] = (a.r1 ? a.r1 : a.r)[l];  // not used without the sweeps
        }
        if (MODE == kGradMasked) e.b[mt] = *reinterpret_cast<const uint2*>(a.below + l * 16 + rg * 4);
    }
}

template <int C, int MODE, int NW>
__device__ __forceinline__ void conv_step(const Geom& g, const ConvArgs& a, const v8s (&wr)[NW],
                                          const float (&bias)[4], float s, const int (&toff)[C == 2 ? 8 : 1],
                                          const int (&doff)[4], int i, int i1, int j0, int k0, int sl,
                                          const EpiIn& cur, EpiIn& nxt,
                                          const lds16* __restrict__ rd, lds16* __restrict__ rq) {
    constexpr int SLOT = slot_u16<C>();
    constexpr bool kLast = MODE == kFinal || MODE == kPrecond;
    const int lane = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int m = lane & 15, rg = lane >> 4;
    const int j = j0 + w;
    const float floor_act = a.relu ? 0.f : -INFINITY;   // hidden activation: max(x, floor)
    const uint32_t keep_all = a.relu ? 0u : 1u;          // input gradient without a ReLU mask
    const int64_t row = ((int64_t)i * g.ny + j) * g.nz;
    __builtin_amdgcn_sched_barrier(0);
    {
        const int p = i + kAhead, sp = ring_next(sl, kAhead + 1);
        dma_plane<C>(a.in, g, p, p <= i1, doff, rq + sp * SLOT);
        if (C == 2 && sp < 2) dma_plane<C>(a.in, g, p, p <= i1, doff, rq + (sp + kRingSlots) * SLOT);
    }
    __builtin_amdgcn_sched_barrier(0);
    epi_load<MODE>(g, a, i + 1, j0, k0, nxt);
    __builtin_amdgcn_sched_barrier(0);
    const float* er = cur.r;
    const float* ed = cur.d;
    const float* er1 = cur.r1;
    const uint8_t* em = cur.m;
    const uint2* eb = cur.b;
    if (j >= g.ny) return;
    int so[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) so[d] = (C == 2 ? sl + d : ring_next(sl, d)) * SLOT;
    if constexpr (kLast) {
        float y[4];
        conv_last_row(rd, so, wr, y);
        if (rg == 0) {
            float out[4];
#pragma unroll
            for (int mt = 0; mt < 4; ++mt) {
                const float v = y[mt] + bias[0];
                if (MODE == kFinal) {
                    out[mt] = v;
                } else {
                    // z = dinv r + C, or between the sweeps z2 = omega dinv r + dinv r1 + C
                    const float di = ed[mt];
                    const float jac = a.r1 ? a.omega * di * er[mt] + di * er1[mt] : di * er[mt];
                    out[mt] = em[mt] ? 0.f : jac + s * sqrtf(di) * v;
                }
            }
            if (k0 + TZ <= g.nz) {
                float* dst = a.out32 + row + k0 + m;
#pragma unroll
                for (int mt = 0; mt < 4; ++mt) dst[16 * mt] = out[mt];
            } else {
#pragma unroll
                for (int mt = 0; mt < 4; ++mt) {
                    const int k = k0 + mt * 16 + m;
                    float* dst = k < g.nz ? a.out32 + row + k : reinterpret_cast<float*>(g_trash) + lane;
                    *dst = out[mt];
                }
            }
        }
    } else {
        // the row as a buffer of nz cells: the stores of lanes past its end
        // fall outside the buffer's range and are dropped
        const __amdgpu_buffer_rsrc_t orow = __builtin_amdgcn_make_buffer_rsrc(a.out16 + row * 16, 0, g.nz * 32, kBufWord3);
        const int vo = (k0 + m) * 32 + rg * 8;  // bytes: cell k0 + m, channels 4 rg..4 rg + 3
        // epilogue of one 16-cell tile mt of the row: bias + activation (or the
        // input gradient's ReLU mask), BF16, one 8-byte store per lane
        auto epi = [&](int mt, const v4f& acc) {
            float h[4];
            // Both epilogues are branch-free: hipcc (ROCm 7.2) miscompiled a
            // per-lane select between the accumulator and 0 written with a
            // branch here (the accumulator register was cleared on every lane).
            if (MODE == kHiddenRelu) {
                // (the first layer's products times the input scale: a power of
                // two, so this equals the products of the scaled input exactly)
#pragma unroll
                for (int q = 0; q < 4; ++q) h[q] = fmaxf((C == 2 ? acc[q] * s : acc[q]) + bias[q], floor_act);
            } else {
                const uint2 bl = eb[mt];
                // ReLU mask: keep the gradient where the activation below is > 0
                // (positive BF16 values are positive as signed 16-bit integers)
                const uint32_t bw[4] = {bl.x << 16, bl.x & 0xffff0000u, bl.y << 16, bl.y & 0xffff0000u};
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const uint32_t pos = (uint32_t)((int32_t)bw[q] > 0);
                    const uint32_t keep = 0u - (pos | keep_all);
                    h[q] = __uint_as_float(__float_as_uint(acc[q]) & keep);
                }
            }
            const u32x2 out = {pack_bf2(h[0], h[1]), pack_bf2(h[2], h[3])};
            // 16 cells further per tile; the next layer reads these from
            // memory: streaming (nontemporal) stores
            __builtin_amdgcn_raw_buffer_store_b64(out, orow, vo + 512 * mt, 0, kNonTemporal);
        };
        if constexpr (C == 16) {
            conv_row16(rd, so, wr, k0 > 0, k0 + TZ < g.nz, epi);
        } else {
            v4f acc[4];
            conv_row2(rd + so[0], toff, wr, acc);
#pragma unroll
            for (int mt = 0; mt < 4; ++mt) epi(mt, acc[mt]);
        }
    }
}

// grid: ncols * ceil(nx / run) blocks of kThreads; at most 168 VGPRs, three
// waves per SIMD.
template <int C, int MODE>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(3))) void conv3d(Geom g, ConvArgs a) {
    // 2-channel input: the ring's slots 0 and 1 are mirrored past its end, so
    // that planes i-1, i, i+1 always sit in three consecutive slots
    if (a.done && *a.done) return;  // the CG loop has ended (the flag is the same for all threads)
    constexpr int kSlots = C == 2 ? kRingSlots + 2 : kRingSlots;
    constexpr int SLOT = slot_u16<C>();
    __shared__ __attribute__((aligned(16))) uint16_t lds[kSlots * SLOT];
    lds16* ring = (lds16*)lds;
    const int lane = threadIdx.x & 63;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int rg = lane >> 4;
    // XCD-aware order: blocks are dealt to the 8 XCDs in turn; block b takes
    // work item x q + min(x, rem) + b / 8 (x = b % 8), so each XCD marches a
    // contiguous range of columns and the y halo rows its neighbours share are
    // found in its own L2
    const int nb = gridDim.x, b = blockIdx.x;
    const int xcd = b & 7, nq = nb >> 3, nrem = nb & 7;
    const int item = xcd * nq + min(xcd, nrem) + (b >> 3);
    const int col = item % a.ncols, chunk = item / a.ncols;
    const int j0 = (col / a.ntk) * TY, k0 = (col % a.ntk) * TZ;
    const int i0 = chunk * a.run;
    const int i1 = min(g.nx, i0 + a.run);
    const int j = j0 + w;
    constexpr bool kLast = MODE == kFinal || MODE == kPrecond;
    constexpr int NW = kLast ? kPairs : (C == 16 ? 3 * kPairs - 1 : 2);
    v8s wr[NW];
#pragma unroll
    for (int t = 0; t < NW; ++t) wr[t] = a.W[t * 64 + lane];
    float bias[4] = {0.f, 0.f, 0.f, 0.f};
    if (MODE == kHiddenRelu) {
#pragma unroll
        for (int q = 0; q < 4; ++q) bias[q] = a.bias[rg * 4 + q];
    } else if (MODE == kFinal || MODE == kPrecond) {
        bias[0] = a.bias[0];
    }
    // kPrecond: the output scale s; first layer: the input scale (1 if none)
    const float s = (MODE == kPrecond) ? *a.sscale
                  : (C == 2 && MODE == kHiddenRelu && a.in_scale) ? *a.in_scale : 1.f;
    int toff[C == 2 ? 8 : 1] = {0};
    if constexpr (C == 2) tap_offsets2(toff);
    // the weights and scalars above have arrived before any plane is requested:
    // no wait inside the march then counts them
    wait_vmcnt(0);
    EpiIn epi;
    epi_load<MODE>(g, a, i0, j0, k0, epi);
    int doff[4];
    dma_offsets<C>(g, j0, k0, doff);
    // the planes i0-1 .. i0+kAhead-1 into slots 0 .. kAhead
#pragma unroll
    for (int d = 0; d <= kAhead; ++d) {
        dma_plane<C>(a.in, g, i0 - 1 + d, i0 - 1 + d <= i1, doff, ring + d * SLOT);
        if (C == 2 && d < 2) dma_plane<C>(a.in, g, i0 - 1 + d, i0 - 1 + d <= i1, doff, ring + (d + kRingSlots) * SLOT);
    }
    // Memory operations of this wave, counted from the kernel start: kq per
    // plane request (a lower bound: the mirror copies are not counted) and,
    // per step, ks stores; the epilogue loads are not counted either. Every
    // count used below is at most the true number, so waiting until at most
    // (issued now - issued up to a plane's request) operations are in flight
    // always covers that request.
    const int kq = dma_per_plane<C>(w);
    const int ks = j < g.ny ? 4 : 0;
    auto issued_through = [&](int p) {  // operations up to and including plane p's request
        const int d = p - i0 + 1;
        return d <= kAhead ? (d + 1) * kq : (kAhead + 1) * kq + (p - kAhead - i0) * (kq + ks) + kq;
    };
    wait_vmcnt((kAhead + 1) * kq - issued_through(i0 + 1));
    ring_barrier();
    int sl = 0;  // slot of plane i - 1
    // plane i + 2 must have arrived, in every wave, before the barrier that ends step i
    auto end_step = [&](int i) {
        wait_vmcnt((kAhead + 1) * kq + (i - i0 + 1) * (kq + ks) - issued_through(i + 2));
        ring_barrier();
        sl = ring_next(sl, 1);
    };
    // two steps per trip: the epilogue operands alternate between two register
    // sets instead of being copied (a copy would wait for the loads at once)
    EpiIn epi2;
#pragma unroll 1
    for (int i = i0; i < i1; i += 2) {
        conv_step<C, MODE>(g, a, wr, bias, s, toff, doff, i, i1, j0, k0, sl, epi, epi2, ring, ring);
        end_step(i);
        if (i + 1 < i1) {
            conv_step<C, MODE>(g, a, wr, bias, s, toff, doff, i + 1, i1, j0, k0, sl, epi2, epi, ring, ring);
            end_step(i + 1);
        }
    }
    wait_vmcnt(0);  // no LDS request outlives the block
}

// The network's scale of a residual from the partials pb of its
// dinv-weighted square (one block, fixed order): scale[0] = s =
// sqrt(sum(dinv r^2) / n_U), scale[1] = 1 / s (both 0 for a zero residual).
__global__ __launch_bounds__(kThreads) void nn_scale(const float* pb, int nb, float n_u, float* scale,
                                                     const int* done) {
    // the first batch of partials in flight with the read of the loop's done flag
    const float* pp[1] = {pb};
    const int np[1] = {nb};
    float first[1][kPartBatch];
    load_partials_first(pp, np, first);
    if (done && block_uniform(early_load(done))) {  // the CG loop has ended
        drain_loads();
        return;
    }
    __shared__ float red[kThreads / kWave];
    float rrs[1];
    sum_partials_n_rest(pp, np, first, red, rrs);
    const float rr = rrs[0];
    if (threadIdx.x == 0) {
        // the power of two nearest the RMS: 2^e with e = floor(log2(rms sqrt 2))
        const int e = rr > 0.f ? ilogbf(sqrtf(rr / n_u) * 1.41421356f) : 0;
        scale[0] = rr > 0.f ? ldexpf(1.f, e) : 0.f;
        scale[1] = rr > 0.f ? ldexpf(1.f, -e) : 0.f;
    }
}

// Network input channels (rh, rh * feat) in BF16. For inference rh is the
// Jacobi-scaled residual sqrt(dinv) r / s (inv_s: the device scalar 1 / s);
// for training (dinv NULL) rh = r is given already scaled. Four cells per
// thread where n allows (every array is 16-byte aligned).
__global__ __launch_bounds__(kThreads) void nn_input(int64_t n, const float* r, const float* dinv,
                                                     const float* feat, const float* inv_s_dev, uint16_t* x0,
                                                     const uint8_t* dmask, const int* done) {
    if (done && *done) return;  // the CG loop has ended
    const float inv_s = inv_s_dev ? *inv_s_dev : 1.f;
    const int64_t stride = (int64_t)gridDim.x * kThreads;
    auto one = [&](float rv, float dv, float fv, bool masked) -> uint32_t {
        float rh = dinv ? sqrtf(dv) * rv * inv_s : rv;
        if (masked) rh = 0.f;
        return pack_bf2(rh, rh * fv);
    };
    int64_t l0 = 0;
    if (n % 4 == 0) {
        for (int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x; e < n / 4; e += stride) {
            const float4 rv = reinterpret_cast<const float4*>(r)[e];
            const float4 fv = reinterpret_cast<const float4*>(feat)[e];
            const float4 dv = dinv ? reinterpret_cast<const float4*>(dinv)[e] : make_float4(1.f, 1.f, 1.f, 1.f);
            const uint32_t mk = dmask ? reinterpret_cast<const uint32_t*>(dmask)[e] : 0u;
            reinterpret_cast<uint4*>(x0)[e] =
                make_uint4(one(rv.x, dv.x, fv.x, mk & 0xffu), one(rv.y, dv.y, fv.y, mk & 0xff00u),
                           one(rv.z, dv.z, fv.z, mk & 0xff0000u), one(rv.w, dv.w, fv.w, mk & 0xff000000u));
        }
        l0 = n;
    }
    for (int64_t l = l0 + (int64_t)blockIdx.x * kThreads + threadIdx.x; l < n; l += stride)
        reinterpret_cast<uint32_t*>(x0)[l] = one(r[l], dinv ? dinv[l] : 1.f, feat[l], dmask && dmask[l]);
}

// The damped Jacobi sweeps around the network (elementwise parts; the
// operator's applies run between them).
// t = omega dinv r on unknown cells, 0 on Dirichlet cells.
__global__ __launch_bounds__(kThreads) void sweep_scale(int64_t n, const float* r, const float* dinv,
                                                        const uint8_t* dmask, float omega, float* t) {
    const int64_t stride = (int64_t)gridDim.x * kThreads;
    for (int64_t l = (int64_t)blockIdx.x * kThreads + threadIdx.x; l < n; l += stride)
        t[l] = dmask[l] ? 0.f : omega * dinv[l] * r[l];
}

// r1 = r - y on unknown cells (y = A t), 0 on Dirichlet cells; per-block
// partial sums of dinv r1^2 (the network's scale of r1).
__global__ __launch_bounds__(kThreads) void sweep_resid(int64_t n, const float* r, const float* y,
                                                        const float* dinv, const uint8_t* dmask, float* r1,
                                                        float* part) {
    __shared__ float red[kThreads / kWave];
    float sum = 0.f;
    const int64_t stride = (int64_t)gridDim.x * kThreads;
    for (int64_t l = (int64_t)blockIdx.x * kThreads + threadIdx.x; l < n; l += stride) {
        const float v = dmask[l] ? 0.f : r[l] - y[l];
        r1[l] = v;
        sum += dinv[l] * v * v;
    }
    const float t = block_sum(sum, red);
    if (threadIdx.x == 0) part[blockIdx.x] = t;
}

// z = z2 + omega dinv (r - y) on unknown cells (y = A z2, held in z on entry),
// 0 on Dirichlet cells.
__global__ __launch_bounds__(kThreads) void sweep_post(int64_t n, const float* z2, const float* r,
                                                       const float* dinv, const uint8_t* dmask, float omega,
                                                       float* z) {
    const int64_t stride = (int64_t)gridDim.x * kThreads;
    for (int64_t l = (int64_t)blockIdx.x * kThreads + threadIdx.x; l < n; l += stride)
        z[l] = dmask[l] ? 0.f : z2[l] + omega * dinv[l] * (r[l] - z[l]);
}

// Weight gradient of one layer over all cells: per-block partial D[t][ci][co]
// (27 x 16 x 16) and bias-gradient partials. Wave w handles taps w, w+4, ...
template <int CIN, int CDY>
__global__ __launch_bounds__(kThreads) void conv_wgrad(Geom g, const uint16_t* __restrict__ x,
                                                       const uint16_t* __restrict__ dy, int ntj,
                                                       int ntk, int ntiles, float* part, float* dbpart) {
    __shared__ __attribute__((aligned(16))) uint16_t lx[HCELLS * CIN];
    __shared__ __attribute__((aligned(16))) uint16_t ld[TY * TZ * 16];
    __shared__ float dbs[kThreads / kWave][16];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int rc = lane & 15, kg = lane >> 4;
    v4f acc[7];
#pragma unroll
    for (int i = 0; i < 7; ++i) acc[i] = v4f{0.f, 0.f, 0.f, 0.f};
    float db[16];
#pragma unroll
    for (int c = 0; c < 16; ++c) db[c] = 0.f;
    for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const Tile T = tile_of(t, ntj, ntk);
        __syncthreads();
        load_halo<CIN>(x, g, T, lx);
        {   // output-gradient tile, no halo; thread = cell of the tile
            const int c = threadIdx.x, yy = c / TZ, zz = c % TZ;
            const int j = T.j0 + yy, k = T.k0 + zz;
            const bool in = j < g.ny && k < g.nz;
            const int64_t l = ((int64_t)T.i * g.ny + j) * g.nz + k;
#pragma unroll
            for (int ch = 0; ch < 16; ++ch) {
                uint16_t v = 0;
                if (in && ch < CDY) v = dy[l * CDY + ch];
                ld[c * 16 + ch] = v;
                db[ch] += bf2f(v);
            }
        }
        __syncthreads();
#pragma unroll
        for (int ti = 0; ti < 7; ++ti) {
            const int tap = w + 4 * ti;
            if (tap >= 27) break;
            const int dx = tap / 9 - 1, dyo = (tap / 3) % 3 - 1, dz = tap % 3 - 1;
            for (int kc = 0; kc < TY * TZ / 16; ++kc) {
                v4s A, B;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int c = kc * 16 + kg * 4 + q;
                    const int yy = c / TZ, zz = c % TZ;
                    const int cell = hcell(1 + dx, yy + 1 + dyo, zz + 1 + dz);
                    const short av = (rc < CIN) ? (short)lx[cell * CIN + rc] : (short)0;
                    const short bv = (short)ld[c * 16 + rc];
                    if (q == 0) { A.x = av; B.x = bv; }
                    if (q == 1) { A.y = av; B.y = bv; }
                    if (q == 2) { A.z = av; B.z = bv; }
                    if (q == 3) { A.w = av; B.w = bv; }
                }
                acc[ti] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(A, B, acc[ti], 0, 0, 0);
            }
        }
    }
    // partials: D[row = ci][col = co], lane holds rows kg*4 + q, column rc
    float* P = part + (size_t)blockIdx.x * 27 * 256;
#pragma unroll
    for (int ti = 0; ti < 7; ++ti) {
        const int tap = w + 4 * ti;
        if (tap >= 27) break;
#pragma unroll
        for (int q = 0; q < 4; ++q) P[tap * 256 + (kg * 4 + q) * 16 + rc] = acc[ti][q];
    }
    // bias gradient: per-thread sums, then waves, then block
#pragma unroll
    for (int c = 0; c < 16; ++c) {
        const float s = wave_sum(db[c]);
        if (lane == 0) dbs[w][c] = s;
    }
    __syncthreads();
    if (threadIdx.x < 16) {
        float s = 0.f;
        for (int i = 0; i < kThreads / kWave; ++i) s += dbs[i][threadIdx.x];
        dbpart[(size_t)blockIdx.x * 16 + threadIdx.x] = s;
    }
}

// Sum the weight-gradient partials of one layer into the FP32 gradient vector.
__global__ void reduce_wgrad(const float* part, const float* dbpart, int nblk, int cin, int cout,
                             float* gW, float* gb) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    const int nw = 27 * cin * cout;
    if (e < nw) {
        const int tap = e / (cin * cout), ci = (e / cout) % cin, co = e % cout;
        const int src = tap * 256 + ci * 16 + co;
        float s = 0.f;
        for (int b = 0; b < nblk; ++b) s += part[(size_t)b * 27 * 256 + src];
        gW[e] = s;
    } else if (e < nw + cout) {
        const int co = e - nw;
        float s = 0.f;
        for (int b = 0; b < nblk; ++b) s += dbpart[(size_t)b * 16 + co];
        gb[co] = s;
    }
}

// Energy-norm loss in the Jacobi-scaled space, z = rh + y on unknown cells.
// With a target t (A~ t = rh): delta = z - t, E = t.rh, loss = delta.A~delta / E.
// Without a target: delta = z, E = rh.rh and the energy functional
// loss = (z.A~z - 2 z.rh) / E, minimal at z = A~^-1 rh (same gradient
// direction, 2 (A~ z - rh) / E). The operator gets w = sqrt(dinv) delta.
__global__ __launch_bounds__(kThreads) void loss_delta(int64_t n, const float* rh, const float* y,
                                                       const float* tgt, const float* dinv,
                                                       const uint8_t* dmask, float* w, float* epart) {
    __shared__ float red[kThreads / kWave];
    float e = 0.f;
    const int64_t stride = (int64_t)gridDim.x * kThreads;
    for (int64_t l = (int64_t)blockIdx.x * kThreads + threadIdx.x; l < n; l += stride) {
        const bool d = dmask[l] != 0;
        const float t = tgt ? tgt[l] : 0.f;
        const float delta = d ? 0.f : rh[l] + y[l] - t;
        w[l] = d ? 0.f : sqrtf(dinv[l]) * delta;
        if (!d) e += (tgt ? t : rh[l]) * rh[l];
    }
    const float tt = block_sum(e, red);
    if (threadIdx.x == 0) epart[blockIdx.x] = tt;
}

// Aw = A (sqrt(dinv) delta), A~ delta = sqrt(dinv) Aw: loss partials and the
// output gradient (first of two BF16 channels).
__global__ __launch_bounds__(kThreads) void loss_grad(int64_t n, const float* rh, const float* y,
                                                      const float* tgt, const float* dinv,
                                                      const uint8_t* dmask, const float* Aw,
                                                      const float* epart, int nb_e, uint16_t* dy,
                                                      float* part) {
    __shared__ float red[kThreads / kWave];
    const float E = sum_partials(epart, nb_e, red);
    const float scale = E > 0.f ? 2.f / E : 0.f;
    float s = 0.f;
    const int64_t stride = (int64_t)gridDim.x * kThreads;
    for (int64_t l = (int64_t)blockIdx.x * kThreads + threadIdx.x; l < n; l += stride) {
        float g = 0.f;
        if (!dmask[l]) {
            const float ad = sqrtf(dinv[l]) * Aw[l];
            const float z = rh[l] + y[l];
            if (tgt) {
                s += (z - tgt[l]) * ad;
                g = scale * ad;
            } else {
                s += z * ad - 2.f * z * rh[l];
                g = scale * (ad - rh[l]);
            }
        }
        reinterpret_cast<uint32_t*>(dy)[l] = (uint32_t)f2bf(g);
    }
    const float t = block_sum(s, red);
    if (threadIdx.x == 0) part[blockIdx.x] = t;
}

// Residual-space loss ||A~ z - rh||^2 / ||rh||^2 (the sparse-approximate-inverse
// objective): after Aw = A (sqrt(dinv) z), g = A~ z - rh is formed and handed
// to the operator again (w2 = sqrt(dinv) g); partials of g.g.
__global__ __launch_bounds__(kThreads) void resid_g(int64_t n, const float* rh, const float* dinv,
                                                    const uint8_t* dmask, const float* Aw, float* w2,
                                                    float* part) {
    __shared__ float red[kThreads / kWave];
    float s = 0.f;
    const int64_t stride = (int64_t)gridDim.x * kThreads;
    for (int64_t l = (int64_t)blockIdx.x * kThreads + threadIdx.x; l < n; l += stride) {
        float g = 0.f;
        if (!dmask[l]) {
            const float sd = sqrtf(dinv[l]);
            g = sd * Aw[l] - rh[l];
            s += g * g;
            g *= sd;
        }
        w2[l] = g;
    }
    const float t = block_sum(s, red);
    if (threadIdx.x == 0) part[blockIdx.x] = t;
}

// dy = 2 A~ g / ||rh||^2 from Ag = A (sqrt(dinv) g).
__global__ __launch_bounds__(kThreads) void resid_grad(int64_t n, const float* dinv,
                                                       const uint8_t* dmask, const float* Ag,
                                                       const float* epart, int nb, uint16_t* dy) {
    __shared__ float red[kThreads / kWave];
    const float E = sum_partials(epart, nb, red);
    const float scale = E > 0.f ? 2.f / E : 0.f;
    const int64_t stride = (int64_t)gridDim.x * kThreads;
    for (int64_t l = (int64_t)blockIdx.x * kThreads + threadIdx.x; l < n; l += stride) {
        const float g = dmask[l] ? 0.f : scale * sqrtf(dinv[l]) * Ag[l];
        reinterpret_cast<uint32_t*>(dy)[l] = (uint32_t)f2bf(g);
    }
}

__global__ __launch_bounds__(kThreads) void loss_final(const float* dpart, const float* epart, int nb,
                                                       double* loss) {
    __shared__ float red[kThreads / kWave];
    const float D = sum_partials(dpart, nb, red);
    const float E = sum_partials(epart, nb, red);
    if (threadIdx.x == 0) *loss = E > 0.f ? (double)D / (double)E : 0.0;
}

__device__ __forceinline__ bool is_bias(int i) {
    for (int l = 0; l < 4; ++l)
        if (i >= offB(l) && i < offB(l) + kCout[l]) return true;
    return false;
}

// Adam on the FP32 master weights; the biases stay fixed (the network output
// then vanishes with its input).
__global__ void adam_kernel(int np, float* p, const float* gr, float* m, float* v, float lr,
                            float b1, float b2, float eps, float bc1, float bc2) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= np || is_bias(i)) return;
    const float g = gr[i];
    const float mi = b1 * m[i] + (1.f - b1) * g;
    const float vi = b2 * v[i] + (1.f - b2) * g * g;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
}

// BF16 operand layouts from the FP32 master weights: one thread per (operand,
// lane), 8 values each (A row i = lane % 16, k = 8 (lane / 16) + v).
__global__ void prepare_weights(const float* p, v8s* W) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= kWTotal) return;
    const int lane = idx & 63, i = lane & 15, q = lane >> 4;
    v8s out;
    for (int v = 0; v < 8; ++v) {
        const int k = 8 * q + v;
        float x = 0.f;
        if (idx < kWf2 || (idx >= kWb4 && idx < kWb3)) {          // 2-channel input, K = 64
            const bool fwd = idx < kWf2;
            const int s = (idx - (fwd ? kWf1 : kWb4)) / 64, kk = 32 * s + k, tap = kk >> 1, ch = kk & 1;
            if (tap < 27) {
                if (fwd) x = p[offW(0) + (tap * 2 + ch) * 16 + i];              // W1[tap][ch][i]
                else if (ch == 0) x = p[offW(3) + (26 - tap) * 16 + i];         // W4[26 - tap][i][0]
            }
        } else if (idx < kWf4 || idx >= kWb3) {                    // 16 -> 16, pair x dz
            const bool fwd = idx < kWf4;
            const int l = fwd ? (idx < kWf3 ? 1 : 2) : (idx < kWb2 ? 2 : 1);
            const int base = fwd ? (l == 1 ? kWf2 : kWf3) : (l == 2 ? kWb3 : kWb2);
            const int op = (idx - base) / 64, P = op / 3, d = op % 3;
            int tap = -1, c = k & 15;
            if (P < kPairs - 1) {
                tap = 3 * (2 * P + (k >> 4)) + d;            // group 2P + (k >> 4), dz = d - 1
            } else if (d == 0) {
                tap = 24 + (k >> 4);                         // group 8: [dz = -1 | dz = 0]
            } else if (d == 1 && k < 16) {
                tap = 26;                                    // group 8: [dz = +1 | 0]
            }                                                // (operand 14 is unused: zeros)
            if (tap >= 0)
                x = fwd ? p[offW(l) + (tap * 16 + c) * 16 + i]                  // W[tap][c][i]
                        : p[offW(l) + ((26 - tap) * 16 + i) * 16 + c];         // W[26 - tap][i][c]
        } else {                                                   // layer 4 forward: rows = dz + 1
            const int P = (idx - kWf4) / 64;
            const int g = 2 * P + (k >> 4), c = k & 15;
            if (g < 9 && i < 3) x = p[offW(3) + ((3 * g + i) * 16 + c)];        // W4[3 g + i][c][0]
        }
        out[v] = (short)f2bf(x);
    }
    W[idx] = out;
}

// log-diagonal feature: log(d) - mean_U log(d) on unknown cells, 0 on Dirichlet
__global__ __launch_bounds__(kThreads) void logd_partials(int64_t n, const float* dinv,
                                                          const uint8_t* dmask, float* part) {
    __shared__ float red[kThreads / kWave];
    float s = 0.f;
    const int64_t stride = (int64_t)gridDim.x * kThreads;
    for (int64_t l = (int64_t)blockIdx.x * kThreads + threadIdx.x; l < n; l += stride)
        if (!dmask[l]) s -= logf(dinv[l]);
    const float t = block_sum(s, red);
    if (threadIdx.x == 0) part[blockIdx.x] = t;
}

__global__ __launch_bounds__(kThreads) void feature_kernel(int64_t n, const float* dinv,
                                                           const uint8_t* dmask, const float* part,
                                                           int nb, float n_u, float* feat, float* sqd) {
    __shared__ float red[kThreads / kWave];
    const float mean = sum_partials(part, nb, red) / n_u;
    const int64_t stride = (int64_t)gridDim.x * kThreads;
    for (int64_t l = (int64_t)blockIdx.x * kThreads + threadIdx.x; l < n; l += stride) {
        feat[l] = dmask[l] ? 0.f : -logf(dinv[l]) - mean;
        sqd[l] = dmask[l] ? 0.f : sqrtf(dinv[l]);
    }
}

int nblocks_for(int64_t n, int cap) {
    int64_t b = (n + kThreads - 1) / kThreads;
    return (int)(b < 1 ? 1 : (b > cap ? cap : b));
}

}  // namespace
}  // namespace mffv

using namespace mffv;

namespace {
std::atomic<int> g_ws_serial{0};
// A positive value never handed out before in this process (wraps after 2^31
// - 1 reallocations, far beyond any run).
int next_ws_serial() {
    int v = g_ws_serial.fetch_add(1) + 1;
    return v > 0 ? v : 1;
}
}  // namespace

struct mffv_net {
    float* params = nullptr;  // FP32 master weights, kNParams
    float* grads = nullptr;
    float* m = nullptr;
    float* v = nullptr;
    v8s* W = nullptr;         // BF16 operand layouts
    int step = 0;             // Adam steps taken
    // activation workspace, sized for `cap` cells
    int64_t cap = 0;
    uint16_t* x0 = nullptr;   // 2 channels
    uint16_t* h1 = nullptr;   // 16 channels each
    uint16_t* h2 = nullptr;
    uint16_t* h3 = nullptr;
    uint16_t* g1 = nullptr;   // output gradients (16 channels)
    uint16_t* g2 = nullptr;
    uint16_t* dy4 = nullptr;  // 2 channels
    float* y = nullptr;
    float* sw1 = nullptr;     // inference: the Jacobi sweeps' vectors (FP32 cells)
    float* sw2 = nullptr;
    float* swp = nullptr;     // per-block partials of the first sweep (swp_cap of them)
    float* swf = nullptr;     // per-block partials of the flexible-CG dots, [4][swp_cap]
    int64_t swp_cap = 0;
    float* t1 = nullptr;      // training scratch (FP32 cells)
    float* t2 = nullptr;
    float* part = nullptr;    // weight-gradient partials
    float* dbpart = nullptr;
    float* red = nullptr;     // reduction partials
    float* sscale = nullptr;
    double* loss = nullptr;
    int wg_blocks = 0;
    bool training_ws = false;
    // identifies the network and its workspace for the solver's captured graphs:
    // a fresh value, unique in the process, at creation and whenever the
    // workspace is reallocated or a flag baked into kernel arguments changes,
    // so that a graph captured with another (possibly destroyed) network at
    // the same address is never replayed
    int ws_gen = 0;
    int relu = 1;             // activation of the hidden layers
    int loss_kind = 0;        // 0 energy norm / functional, 1 residual space
};

namespace {

int nfail(int code, const std::string& m) { return set_error(code, m); }

template <class T>
int nalloc(T** p, size_t count) {
    if (hipMalloc(reinterpret_cast<void**>(p), count * sizeof(T)) != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        return MFFV_ENOMEM;
    }
    return MFFV_OK;
}
template <class T>
void nfree(T*& p) {
    if (p) (void)hipFree(p);
    p = nullptr;
}

constexpr int kRedBlocks = 1024;
constexpr int kFlexBlocks = 1024;  // target count of the fused flexible-CG dot partials

void free_ws(mffv_net* N) {
    nfree(N->x0); nfree(N->h1); nfree(N->h2); nfree(N->h3); nfree(N->g1); nfree(N->g2);
    nfree(N->dy4); nfree(N->y); nfree(N->t1); nfree(N->t2); nfree(N->sw1); nfree(N->sw2); nfree(N->swp); nfree(N->swf);
    N->cap = 0;
    N->swp_cap = 0;
    N->training_ws = false;
}

int ensure_ws(mffv_net* N, int64_t n, bool training) {
    if (n <= N->cap && (!training || N->training_ws)) return MFFV_OK;
    const int64_t cap = std::max<int64_t>(n, N->cap);
    free_ws(N);
    N->ws_gen = next_ws_serial();
    int rc;
    if ((rc = nalloc(&N->x0, (size_t)cap * 2)) || (rc = nalloc(&N->h1, (size_t)cap * 16)) ||
        (rc = nalloc(&N->h2, (size_t)cap * 16)) || (rc = nalloc(&N->y, (size_t)cap)) ||
        (rc = nalloc(&N->sw1, (size_t)cap)) || (rc = nalloc(&N->sw2, (size_t)cap)) ||
        (rc = nalloc(&N->swp, (size_t)(cap / 256 + 8192))) || (rc = nalloc(&N->swf, 4 * (size_t)(cap / 256 + 8192)))) {
        free_ws(N);
        return nfail(rc, "network workspace allocation failed");
    }
    // a stencil launch has at most about n / 256 + nx blocks; grids with more
    // (very many thin planes) take the unfused sweeps
    N->swp_cap = cap / 256 + 8192;
    if (training) {
        if ((rc = nalloc(&N->h3, (size_t)cap * 16)) || (rc = nalloc(&N->g1, (size_t)cap * 16)) ||
            (rc = nalloc(&N->g2, (size_t)cap * 16)) || (rc = nalloc(&N->dy4, (size_t)cap * 2)) ||
            (rc = nalloc(&N->t1, (size_t)cap)) || (rc = nalloc(&N->t2, (size_t)cap))) {
            free_ws(N);
            return nfail(rc, "network training workspace allocation failed");
        }
        N->training_ws = true;
    }
    N->cap = cap;
    return MFFV_OK;
}

#define NHIP(expr)                                                              \
    do {                                                                        \
        hipError_t e_ = (expr);                                                 \
        if (e_ != hipSuccess) return nfail(MFFV_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

struct Shape {
    Geom g;
    int ntj, ntk, ntiles;
};

Shape shape_of(int nx, int ny, int nz) {
    Shape s;
    s.g = Geom{nx, ny, nz, (int64_t)nx * ny * nz, (int64_t)ny * nz};
    s.ntj = (ny + TY - 1) / TY;
    s.ntk = (nz + TZ - 1) / TZ;
    s.ntiles = nx * s.ntj * s.ntk;
    return s;
}

// Blocks of a kernel that fit on the device at once (CUs x resident blocks per CU).
template <class K>
int64_t resident_blocks(K kernel) {
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, kThreads, 0) != hipSuccess)
        return 768;
    return std::max<int64_t>(1, (int64_t)cus * per_cu);
}

// x planes per block of the marching convolution: the shortest run for which
// all blocks are resident at once (one round, no tail), but at least two
// planes, so the two halo planes of a run cost at most one plane per output plane.
int conv_run(const Shape& S, int64_t slots) {
    const int64_t cols = (int64_t)S.ntj * S.ntk;
    int64_t run = (S.g.nx * cols + slots - 1) / slots;
    run = std::max<int64_t>(run, 2);
    return (int)std::min<int64_t>(run, S.g.nx);
}

// Planes per block set by mffv_set_nn_run (0: conv_run's choice).
int g_nn_run = 0;

template <int C, int MODE>
int conv(const Shape& S, const ConvArgs& a0, hipStream_t st) {
    static const int64_t slots = resident_blocks(conv3d<C, MODE>);
    ConvArgs a = a0;
    a.ntk = S.ntk;
    a.ncols = S.ntj * S.ntk;
    a.run = g_nn_run > 0 ? std::min(g_nn_run, S.g.nx) : conv_run(S, slots);
    const int64_t blocks = (int64_t)a.ncols * ((S.g.nx + a.run - 1) / a.run);
    hipLaunchKernelGGL((conv3d<C, MODE>), dim3((unsigned)blocks), dim3(kThreads), 0, st, S.g, a);
    NHIP(hipGetLastError());
    return MFFV_OK;
}

// Forward through the four layers from N->x0 (already filled); the last layer
// either stores y (training) or forms the preconditioned z. keep_h3
// (training) keeps h3 for the backward pass; inference writes it over h1.
int forward(mffv_net* N, const Shape& S, bool keep_h3, int last_mode, const ConvArgs& last,
            hipStream_t st, hipEvent_t* ev = nullptr, const int* done = nullptr,
            const float* in_scale = nullptr) {
    if (ev) NHIP(hipEventRecord(ev[0], st));
    ConvArgs a{};
    a.done = done;
    a.in_scale = in_scale;
    a.relu = N->relu;
    a.in = N->x0;
    a.W = N->W + kWf1;
    a.bias = N->params + offB(0);
    a.out16 = N->h1;
    int rc;
    if ((rc = conv<2, kHiddenRelu>(S, a, st))) return rc;
    a.in_scale = nullptr;
    if (ev) NHIP(hipEventRecord(ev[1], st));
    a.in = N->h1;
    a.W = N->W + kWf2;
    a.bias = N->params + offB(1);
    a.out16 = N->h2;
    if ((rc = conv<16, kHiddenRelu>(S, a, st))) return rc;
    if (ev) NHIP(hipEventRecord(ev[2], st));
    uint16_t* h3 = keep_h3 ? N->h3 : N->h1;  // inference reuses h1's buffer
    a.in = N->h2;
    a.W = N->W + kWf3;
    a.bias = N->params + offB(2);
    a.out16 = h3;
    if ((rc = conv<16, kHiddenRelu>(S, a, st))) return rc;
    if (ev) NHIP(hipEventRecord(ev[3], st));
    ConvArgs f = last;
    f.done = done;
    f.relu = N->relu;
    f.in = h3;
    f.W = N->W + kWf4;
    f.bias = N->params + offB(3);
    rc = last_mode == kFinal ? conv<16, kFinal>(S, f, st) : conv<16, kPrecond>(S, f, st);
    if (rc) return rc;
    if (ev) NHIP(hipEventRecord(ev[4], st));
    return MFFV_OK;
}

int backward(mffv_net* N, const Shape& S, hipStream_t st) {
    int rc;
    const int nb = N->wg_blocks = std::min(S.ntiles, 512);
    auto wgrad = [&](int layer, const uint16_t* x, const uint16_t* dy) -> int {
        if (layer == 0)
            hipLaunchKernelGGL((conv_wgrad<2, 16>), dim3(nb), dim3(kThreads), 0, st, S.g, x, dy, S.ntj, S.ntk, S.ntiles, N->part, N->dbpart);
        else if (layer == 3)
            hipLaunchKernelGGL((conv_wgrad<16, 2>), dim3(nb), dim3(kThreads), 0, st, S.g, x, dy, S.ntj, S.ntk, S.ntiles, N->part, N->dbpart);
        else
            hipLaunchKernelGGL((conv_wgrad<16, 16>), dim3(nb), dim3(kThreads), 0, st, S.g, x, dy, S.ntj, S.ntk, S.ntiles, N->part, N->dbpart);
        NHIP(hipGetLastError());
        const int tot = 27 * kCin[layer] * kCout[layer] + kCout[layer];
        hipLaunchKernelGGL(reduce_wgrad, dim3((tot + 255) / 256), dim3(256), 0, st, N->part, N->dbpart, nb,
                           kCin[layer], kCout[layer], N->grads + offW(layer), N->grads + offB(layer));
        NHIP(hipGetLastError());
        return MFFV_OK;
    };
    // layer 4: dy4 -> grad of h3 (masked by h3 > 0) into g1
    ConvArgs a{};
    a.relu = N->relu;
    a.in = N->dy4;
    a.W = N->W + kWb4;
    a.out16 = N->g1;
    a.below = N->h3;
    if ((rc = conv<2, kGradMasked>(S, a, st))) return rc;
    if ((rc = wgrad(3, N->h3, N->dy4))) return rc;
    // layer 3: g1 -> grad of h2 into g2
    a.in = N->g1;
    a.W = N->W + kWb3;
    a.out16 = N->g2;
    a.below = N->h2;
    if ((rc = conv<16, kGradMasked>(S, a, st))) return rc;
    if ((rc = wgrad(2, N->h2, N->g1))) return rc;
    // layer 2: g2 -> grad of h1 into g1
    a.in = N->g2;
    a.W = N->W + kWb2;
    a.out16 = N->g1;
    a.below = N->h1;
    if ((rc = conv<16, kGradMasked>(S, a, st))) return rc;
    if ((rc = wgrad(1, N->h1, N->g2))) return rc;
    // layer 1
    return wgrad(0, N->x0, N->g1);
}

int refresh_weights(mffv_net* N, hipStream_t st) {
    hipLaunchKernelGGL(prepare_weights, dim3((kWTotal + 255) / 256), dim3(256), 0, st, N->params, N->W);
    NHIP(hipGetLastError());
    return MFFV_OK;
}

int check_net(const mffv_net* N) {
    if (!N) return nfail(MFFV_EINVAL, "network handle is NULL");
    return MFFV_OK;
}

int check_shape(int nx, int ny, int nz) {
    if (nx < 1 || ny < 1 || nz < 1 || (int64_t)nx * ny * nz >= (int64_t(1) << 31))
        return nfail(MFFV_EINVAL, "bad grid shape");
    return MFFV_OK;
}

// One pass of forward + energy-norm loss (+ backward) for a training pair on
// the operator (g, c). Fills N->loss (device).
int loss_pass(mffv_net* N, const Shape& S, const Coef& c, const March& m, const float* dinv,
              const uint8_t* dmask, const float* feat, const float* r_hat, const float* target,
              bool grads, hipStream_t st) {
    int rc;
    const int64_t n = S.g.n;
    const int nb = nblocks_for(n, kRedBlocks);
    hipLaunchKernelGGL(nn_input, dim3(nb), dim3(kThreads), 0, st, n, r_hat, (const float*)nullptr, feat,
                       (const float*)nullptr, N->x0, dmask, (const int*)nullptr);
    NHIP(hipGetLastError());
    ConvArgs last{};
    last.out32 = N->y;
    if ((rc = forward(N, S, true, kFinal, last, st))) return rc;
    if (N->loss_kind == 1) {
        // residual space: w = sqrt(dinv) z, Aw, g = A~ z - rh, w2 = sqrt(dinv) g, A w2
        hipLaunchKernelGGL(loss_delta, dim3(nb), dim3(kThreads), 0, st, n, r_hat, (const float*)N->y,
                           (const float*)nullptr, dinv, dmask, N->t1, N->red);  // E = rh.rh
        NHIP(hipGetLastError());
        StencilIO<float> io;
        io.src = N->t1;
        io.out = N->t2;
        NHIP(launch_stencil_f32(kApply, S.g, c, io, m, st));
        hipLaunchKernelGGL(resid_g, dim3(nb), dim3(kThreads), 0, st, n, r_hat, dinv, dmask,
                           (const float*)N->t2, N->t1, N->red + kRedBlocks);
        NHIP(hipGetLastError());
        io.src = N->t1;
        io.out = N->t2;
        NHIP(launch_stencil_f32(kApply, S.g, c, io, m, st));
        hipLaunchKernelGGL(resid_grad, dim3(nb), dim3(kThreads), 0, st, n, dinv, dmask, (const float*)N->t2,
                           (const float*)N->red, nb, N->dy4);
        NHIP(hipGetLastError());
    } else {
        hipLaunchKernelGGL(loss_delta, dim3(nb), dim3(kThreads), 0, st, n, r_hat, (const float*)N->y, target, dinv,
                           dmask, N->t1, N->red);
        NHIP(hipGetLastError());
        StencilIO<float> io;
        io.src = N->t1;
        io.out = N->t2;
        NHIP(launch_stencil_f32(kApply, S.g, c, io, m, st));
        hipLaunchKernelGGL(loss_grad, dim3(nb), dim3(kThreads), 0, st, n, r_hat, (const float*)N->y, target, dinv,
                           dmask, (const float*)N->t2, (const float*)N->red, nb, N->dy4, N->red + kRedBlocks);
        NHIP(hipGetLastError());
    }
    hipLaunchKernelGGL(loss_final, dim3(1), dim3(kThreads), 0, st, (const float*)(N->red + kRedBlocks),
                       (const float*)N->red, nb, N->loss);
    NHIP(hipGetLastError());
    if (grads) return backward(N, S, st);
    return MFFV_OK;
}

}  // namespace

namespace mffv {

int nn_precondition(const mffv_net* Nc, const Geom& g, const Coef& c, const March& m, float omega,
                    const float* r, const float* dinv, const uint8_t* dmask, const float* sqd, float* z,
                    const float* pb, int nb_b, const float* feat, float n_u, hipStream_t s,
                    const float* q, const float** flex_part, int* nb_flex, hipEvent_t* layer_ev,
                    const int* done) {
    *flex_part = nullptr;
    *nb_flex = 0;
    mffv_net* N = const_cast<mffv_net*>(Nc);
    if (g.n > N->cap) return nfail(MFFV_ESTATE, "network workspace not prepared for this grid");
    const Shape S = shape_of(g.nx, g.ny, g.nz);
    const int nb = nblocks_for(g.n, kRedBlocks);
    const float* rin = r;    // the residual the network sees
    const float* pin = pb;   // and the partials of its dinv-weighted square
    int nbin = nb_b;
    // the sweeps as single passes over the operator (kSweep1 / kSweep2 of the
    // stencil kernels) when the first one's partials fit
    const bool fused = (int64_t)m.blocks() <= N->swp_cap;
    if (omega > 0.f && fused) {
        // first sweep: r1 = r - A (omega dinv r), with the partials of dinv r1^2;
        // r1 itself goes out only as the network's unscaled BF16 input
        // (sqrt(dinv) r1, sqrt(dinv) r1 f), the first convolution applying 1/s
        StencilIO<float> io;
        io.src = r;
        io.dinv = dinv;
        io.omega = omega;
        io.out = nullptr;
        io.nn_x0 = reinterpret_cast<uint32_t*>(N->x0);
        io.nn_feat = feat;
        io.partials = N->swp;
        io.sw_j = N->sw2;   // omega dinv r + dinv r1, for z2
        io.done = done;
        NHIP(launch_stencil_f32(kSweep1, g, c, io, m, s));
        hipLaunchKernelGGL(nn_scale, dim3(1), dim3(kThreads), 0, s, (const float*)N->swp, (int)m.blocks(), n_u,
                           N->sscale, done);
        NHIP(hipGetLastError());
        // the network's output y into N->y; the second sweep's pass forms
        // z2 = (omega dinv r + dinv r1) + s sqrt(dinv) y (0 on Dirichlet cells,
        // where both terms are 0) at every stencil point and writes
        // z = z2 + omega dinv (r - A z2)
        ConvArgs last{};
        last.out32 = N->y;
        int rc = forward(N, S, false, kFinal, last, s, layer_ev, done, N->sscale + 1);
        if (rc) return rc;
        StencilIO<float> io2;
        io2.done = done;
        io2.src = N->y;
        io2.out = z;
        io2.rres = r;
        io2.dinv = dinv;
        io2.omega = omega;
        io2.sw_j = N->sw2;
        io2.sw_sq = sqd;
        io2.sw_scale = N->sscale;
        io2.sw_flex = N->swf;
        io2.sw_q = q;
        // every block of the next phase A sums these partials: at most about
        // kFlexBlocks of them (more planes per block if the plan has more)
        March m2 = m;
        if (m.blocks() > kFlexBlocks) {
            const int f = (m.blocks() + kFlexBlocks - 1) / kFlexBlocks;
            m2 = plan_march(g, m.vec, std::min(g.nx, m.ci * f), m.remap, m.nseg ? m.seg : -1);
        }
        NHIP(launch_stencil_f32(kSweep2, g, c, io2, m2, s));
        *flex_part = N->swf;
        *nb_flex = m2.blocks();
        return MFFV_OK;
    } else if (omega > 0.f) {
        // the same in three kernels: t = omega dinv r into sw1, A t into sw2, r1 into sw1
        hipLaunchKernelGGL(sweep_scale, dim3(nb), dim3(kThreads), 0, s, g.n, r, dinv, dmask, omega, N->sw1);
        NHIP(hipGetLastError());
        StencilIO<float> io;
        io.src = N->sw1;
        io.out = N->sw2;
        NHIP(launch_stencil_f32(kApply, g, c, io, m, s));
        hipLaunchKernelGGL(sweep_resid, dim3(nb), dim3(kThreads), 0, s, g.n, r, (const float*)N->sw2, dinv, dmask,
                           N->sw1, N->red);
        NHIP(hipGetLastError());
        rin = N->sw1;
        pin = N->red;
        nbin = nb;
    }
    hipLaunchKernelGGL(nn_scale, dim3(1), dim3(kThreads), 0, s, pin, nbin, n_u, N->sscale, done);
    NHIP(hipGetLastError());
    hipLaunchKernelGGL(nn_input, dim3(nb), dim3(kThreads), 0, s, g.n, rin, dinv, feat,
                       (const float*)(N->sscale + 1), N->x0, (const uint8_t*)nullptr, done);
    NHIP(hipGetLastError());
    ConvArgs last{};
    last.out32 = omega > 0.f ? N->sw2 : z;   // z2 before the second sweep
    last.r = r;
    last.r1 = omega > 0.f ? N->sw1 : nullptr;
    last.omega = omega;
    last.dinv = dinv;
    last.dmask = dmask;
    last.sscale = N->sscale;
    int rc = forward(N, S, false, kPrecond, last, s, layer_ev);
    if (rc || !(omega > 0.f)) return rc;
    // second sweep: z = z2 + omega dinv (r - A z2)
    StencilIO<float> io;
    io.src = N->sw2;
    io.out = z;
    NHIP(launch_stencil_f32(kApply, g, c, io, m, s));  // A z2 into z, then the update
    hipLaunchKernelGGL(sweep_post, dim3(nb), dim3(kThreads), 0, s, g.n, (const float*)N->sw2, r, dinv, dmask, omega, z);
    NHIP(hipGetLastError());
    return MFFV_OK;
}

int nn_feature(const Geom& g, const float* dinv, const uint8_t* dmask, float n_u, float* part,
               float* feat, float* sqd, hipStream_t s) {
    const int nb = nblocks_for(g.n, kRedBlocks);
    hipLaunchKernelGGL(logd_partials, dim3(nb), dim3(kThreads), 0, s, g.n, dinv, dmask, part);
    NHIP(hipGetLastError());
    hipLaunchKernelGGL(feature_kernel, dim3(nb), dim3(kThreads), 0, s, g.n, dinv, dmask, (const float*)part, nb,
                       n_u, feat, sqd);
    NHIP(hipGetLastError());
    return MFFV_OK;
}

int nn_loss(mffv_net* N, const Geom& g, const Coef& c, const March& m, const float* dinv,
            const uint8_t* dmask, const float* feat, const float* r_hat, const float* target,
            bool grads, hipStream_t st) {
    int rc = ensure_ws(N, g.n, true);
    if (rc) return rc;
    return loss_pass(N, shape_of(g.nx, g.ny, g.nz), c, m, dinv, dmask, feat, r_hat, target, grads, st);
}

int nn_adam(mffv_net* N, float lr, hipStream_t st) {
    N->step += 1;
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    const float bc1 = 1.f - std::pow(b1, (float)N->step), bc2 = 1.f - std::pow(b2, (float)N->step);
    hipLaunchKernelGGL(adam_kernel, dim3((kNParams + 255) / 256), dim3(256), 0, st, kNParams, N->params,
                       (const float*)N->grads, N->m, N->v, lr, b1, b2, eps, bc1, bc2);
    NHIP(hipGetLastError());
    return refresh_weights(N, st);
}

const double* nn_loss_ptr(const mffv_net* N) { return N->loss; }

int nn_prepare(const mffv_net* Nc, int64_t n) {
    mffv_net* N = const_cast<mffv_net*>(Nc);
    const int64_t before = N->cap;
    const void* h1 = N->h1;
    int rc = ensure_ws(N, n, false);
    if (rc) return rc;
    if (N->cap != before || N->h1 != h1) N->ws_gen = next_ws_serial();
    return N->ws_gen;
}

}  // namespace mffv

extern "C" {

int mffv_net_create(const float* params, mffv_net** out) {
    if (!out) return nfail(MFFV_EINVAL, "out is NULL");
    mffv_net* N = new (std::nothrow) mffv_net();
    if (!N) return nfail(MFFV_ENOMEM, "host allocation failed");
    N->ws_gen = next_ws_serial();
    int rc;
    if ((rc = nalloc(&N->params, kNParams)) || (rc = nalloc(&N->grads, kNParams)) ||
        (rc = nalloc(&N->m, kNParams)) || (rc = nalloc(&N->v, kNParams)) ||
        (rc = nalloc(&N->W, kWTotal)) ||
        (rc = nalloc(&N->part, (size_t)512 * 27 * 256)) || (rc = nalloc(&N->dbpart, (size_t)512 * 16)) ||
        (rc = nalloc(&N->red, 2 * (size_t)kRedBlocks)) || (rc = nalloc(&N->sscale, 2)) ||
        (rc = nalloc(&N->loss, 1))) {
        mffv_net_destroy(N);
        return nfail(rc, "network allocation failed");
    }
    std::vector<float> zero(kNParams, 0.f);
    const float* src = params ? params : zero.data();
    for (int i = 0; i < kNParams; ++i)
        if (!std::isfinite(src[i])) {
            mffv_net_destroy(N);
            return nfail(MFFV_EINVAL, "non-finite network parameter");
        }
    if (hipMemcpy(N->params, src, kNParams * sizeof(float), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemset(N->m, 0, kNParams * sizeof(float)) != hipSuccess ||
        hipMemset(N->v, 0, kNParams * sizeof(float)) != hipSuccess ||
        hipMemset(N->grads, 0, kNParams * sizeof(float)) != hipSuccess ||
        refresh_weights(N, nullptr) != MFFV_OK || hipDeviceSynchronize() != hipSuccess) {
        mffv_net_destroy(N);
        return nfail(MFFV_EHIP, "network initialisation failed");
    }
    *out = N;
    return MFFV_OK;
}

void mffv_net_destroy(mffv_net* N) {
    if (!N) return;
    (void)hipDeviceSynchronize();
    free_ws(N);
    nfree(N->params); nfree(N->grads); nfree(N->m); nfree(N->v); nfree(N->W); nfree(N->part);
    nfree(N->dbpart); nfree(N->red); nfree(N->sscale); nfree(N->loss);
    delete N;
}

int mffv_net_num_params(void) { return kNParams; }

int mffv_net_set_loss(mffv_net* N, int kind) {
    int rc = check_net(N);
    if (rc) return rc;
    if (kind != 0 && kind != 1) return nfail(MFFV_EINVAL, "loss kind must be 0 (energy) or 1 (residual)");
    N->loss_kind = kind;
    return MFFV_OK;
}

int mffv_set_nn_run(int run) {
    if (run < 0) return nfail(MFFV_EINVAL, "run must be >= 0");
    g_nn_run = run;
    return MFFV_OK;
}

int mffv_net_set_activation(mffv_net* N, int relu) {
    int rc = check_net(N);
    if (rc) return rc;
    if (relu != 0 && relu != 1) return nfail(MFFV_EINVAL, "activation must be 0 (identity) or 1 (ReLU)");
    NHIP(hipDeviceSynchronize());
    N->relu = relu;
    N->ws_gen = next_ws_serial();  // captured graphs baked the old flag into their kernel arguments
    return MFFV_OK;
}

int mffv_net_get_params(const mffv_net* N, float* params, float* grads) {
    int rc = check_net(N);
    if (rc) return rc;
    if (!params && !grads) return nfail(MFFV_EINVAL, "nothing to copy");
    NHIP(hipDeviceSynchronize());
    if (params) NHIP(hipMemcpy(params, N->params, kNParams * sizeof(float), hipMemcpyDeviceToHost));
    if (grads) NHIP(hipMemcpy(grads, N->grads, kNParams * sizeof(float), hipMemcpyDeviceToHost));
    return MFFV_OK;
}

int mffv_net_set_params(mffv_net* N, const float* params) {
    int rc = check_net(N);
    if (rc) return rc;
    if (!params) return nfail(MFFV_EINVAL, "params is NULL");
    for (int i = 0; i < kNParams; ++i)
        if (!std::isfinite(params[i])) return nfail(MFFV_EINVAL, "non-finite network parameter");
    NHIP(hipDeviceSynchronize());
    NHIP(hipMemcpy(N->params, params, kNParams * sizeof(float), hipMemcpyHostToDevice));
    NHIP(hipMemset(N->m, 0, kNParams * sizeof(float)));
    NHIP(hipMemset(N->v, 0, kNParams * sizeof(float)));
    N->step = 0;
    if ((rc = refresh_weights(N, nullptr))) return rc;
    NHIP(hipDeviceSynchronize());
    return MFFV_OK;
}

int mffv_nn_forward(mffv_net* N, int nx, int ny, int nz, const float* r_hat, const float* feat,
                    float* out, void* stream) {
    int rc;
    if ((rc = check_net(N)) || (rc = check_shape(nx, ny, nz))) return rc;
    if (!r_hat || !feat || !out) return nfail(MFFV_EINVAL, "NULL array");
    const Shape S = shape_of(nx, ny, nz);
    if ((rc = ensure_ws(N, S.g.n, true))) return rc;
    hipStream_t st = static_cast<hipStream_t>(stream);
    hipLaunchKernelGGL(nn_input, dim3(nblocks_for(S.g.n, kRedBlocks)), dim3(kThreads), 0, st, S.g.n, r_hat,
                       (const float*)nullptr, feat, (const float*)nullptr, N->x0,
                       (const uint8_t*)nullptr, (const int*)nullptr);
    NHIP(hipGetLastError());
    ConvArgs last{};
    last.out32 = out;
    return forward(N, S, false, kFinal, last, st);
}

int mffv_nn_time_layers(mffv_net* N, int nx, int ny, int nz, const float* r_hat, const float* feat, int reps,
                        double* us, void* stream) {
    int rc;
    if ((rc = check_net(N)) || (rc = check_shape(nx, ny, nz))) return rc;
    if (!r_hat || !feat || !us) return nfail(MFFV_EINVAL, "NULL array");
    if (reps < 1) return nfail(MFFV_EINVAL, "reps must be >= 1");
    const Shape S = shape_of(nx, ny, nz);
    if ((rc = ensure_ws(N, S.g.n, false))) return rc;
    hipStream_t st = static_cast<hipStream_t>(stream);
    // one whole pass first, so that every layer reads what the network computes
    hipLaunchKernelGGL(nn_input, dim3(nblocks_for(S.g.n, kRedBlocks)), dim3(kThreads), 0, st, S.g.n, r_hat,
                       (const float*)nullptr, feat, (const float*)nullptr, N->x0, (const uint8_t*)nullptr,
                       (const int*)nullptr);
    NHIP(hipGetLastError());
    ConvArgs last{};
    last.out32 = N->y;
    if ((rc = forward(N, S, false, kFinal, last, st))) return rc;
    hipEvent_t ev[2];
    NHIP(hipEventCreate(&ev[0]));
    if (hipEventCreate(&ev[1]) != hipSuccess) {
        (void)hipEventDestroy(ev[0]);
        return nfail(MFFV_EHIP, "hipEventCreate failed");
    }
    rc = MFFV_OK;
    for (int l = 0; l < 4 && rc == MFFV_OK; ++l) {
        ConvArgs a{};
        a.relu = N->relu;
        a.W = N->W + (l == 0 ? kWf1 : l == 1 ? kWf2 : l == 2 ? kWf3 : kWf4);
        a.bias = N->params + offB(l);
        a.in = l == 0 ? N->x0 : l == 1 ? N->h1 : l == 2 ? N->h2 : N->h1;
        a.out16 = l == 0 ? N->h1 : l == 1 ? N->h2 : N->h1;  // inference keeps h3 in h1
        a.out32 = N->y;
        if (hipEventRecord(ev[0], st) != hipSuccess) rc = nfail(MFFV_EHIP, "hipEventRecord failed");
        for (int k = 0; k < reps && rc == MFFV_OK; ++k)
            rc = l == 0 ? conv<2, kHiddenRelu>(S, a, st) : l < 3 ? conv<16, kHiddenRelu>(S, a, st)
                                                                 : conv<16, kFinal>(S, a, st);
        if (rc == MFFV_OK && hipEventRecord(ev[1], st) != hipSuccess) rc = nfail(MFFV_EHIP, "hipEventRecord failed");
        float ms = 0.f;
        if (rc == MFFV_OK && (hipEventSynchronize(ev[1]) != hipSuccess ||
                              hipEventElapsedTime(&ms, ev[0], ev[1]) != hipSuccess))
            rc = nfail(MFFV_EHIP, "event timing failed");
        if (rc == MFFV_OK) us[l] = 1e3 * (double)ms / reps;
    }
    (void)hipEventDestroy(ev[0]);
    (void)hipEventDestroy(ev[1]);
    return rc;
}

}  // extern "C"
