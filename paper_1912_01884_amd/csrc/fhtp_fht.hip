// Band Fast Hough Transform for mostly vertical lines (Section 2.1).
//
// Every band of n = 2^p rows is zero-extended to the right by n columns and
// transformed with the dyadic shift-and-add recursion: stage j merges pairs of
// row blocks of 2^(j-1) rows into blocks of 2^j rows,
//
//   T_j(b, c, s) = T_{j-1}(2b, c, s/2) + T_{j-1}(2b+1, c + ceil(s/2), s/2)   (s/2 rounded down),
//
// so after p stages T_p(0, c, s) is the sum along the dyadic line that starts
// at column c and is displaced by s over the band.  Left-leaning lines are the
// same recursion on the band mirrored about its (cyclic) width, so both
// directions share one code path ("c-space": c = x for right-leaning lines,
// c = W-1-x for left-leaning ones).  Work per band and direction is p*n*W
// additions, the O((w + h/k) * (h/k) * log(h/k)) cost of Section 2.1.
//
// Layout on gfx950: one thread owns one c-space column and keeps the n running
// sums of that column in VGPRs through all p stages; the operand that comes
// from another column (c + ceil(s/2)) is exchanged through LDS once per
// stage.  A workgroup of NT threads covers NC columns (its waves overlap by a
// few columns) and produces the NC - (n-1) leftmost of them (the rest are its
// halo).  Global loads and table
// stores are coalesced along x.  Bands taller than 2^7 rows run the same kernel
// on 128-row sub-blocks, then a second kernel adds the sub-blocks along the
// coarse levels of the recursion.
#include <algorithm>
#include <atomic>
#include <vector>

#include "fhtp_internal.h"

namespace fhtp {
namespace {

// Column offset of row y on the dyadic line of shift s over 2^p rows: bit
// (p-1-j) of y contributes ceil((s >> j) / 2).
__device__ __forceinline__ int dyadic_offset(int p, int s, int y) {
    int off = 0;
    for (int j = 0; j < p; ++j)
        if ((y >> (p - 1 - j)) & 1) off += (s >> (j + 1)) + ((s >> j) & 1);
    return off;
}

// Buffer resource over [base, base + bytes): loads beyond the extent read 0
// and stores beyond it are dropped by the hardware.  The third descriptor
// word selects 32-bit raw (untyped) access on the gfx9 family.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* base, unsigned int bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes,
                                             0x00020000);
}

template <typename PixT>
__device__ __forceinline__ uint32_t buffer_pixel(__amdgpu_buffer_rsrc_t r, unsigned int voff,
                                                 unsigned int soff) {
    if constexpr (sizeof(PixT) == 1)
        return __builtin_amdgcn_raw_buffer_load_b8(r, (int)voff, (int)soff, 0);
    else
        return __builtin_amdgcn_raw_buffer_load_b16(r, (int)voff, (int)soff, 0);
}

// Stages 1 .. kLaneStages take their operands from lanes + 1 .. + 2^(J-1) of
// the wave instead of LDS (stage J reads columns c .. c + 2^(J-1)).
constexpr int kLaneStages = 2;

template <int P>
struct RegCfg {
    static constexpr int N = 1 << P;
    static constexpr int NT = (P >= 7) ? 512 : 256;
    static constexpr int HALF = (N >= 2) ? N / 2 : 1;
    // Distinct columns of a workgroup: consecutive waves overlap by K columns
    // (see from_next_lane), so 64 - K per wave plus the last wave's K.
    static constexpr int K = (P >= 1) ? (1 << kLaneStages) - 1 : 0;
    static constexpr int NC = NT - (NT / 64 - 1) * K;
    // LDS holds the exchanged operands column by column: (column c, row r) at
    // c * RW + r.  RW is odd so that the 64 lanes of a wave, one column each,
    // hit distinct banks.  Reads reach column NC + HALF - 2; column NT + HALF
    // is the spare written by duplicate lanes.
    static constexpr int RW = (HALF >= 2) ? HALF + 1 : 1;
    static constexpr int SPARE = NT + HALF;
    static constexpr int LDS_WORDS = (N >= 2) ? (SPARE + 1) * RW : 1;
    static constexpr int NPK = (N + 1) / 2;            // packed 16-bit pixel pairs per column
    static constexpr int NDIR = (P == 0) ? 1 : 2;      // one-row bands have only d = 0
    // Fetch the next item's pixels during the current item's stages.  At
    // n = 128 the 128 running sums leave no registers for it.
    static constexpr bool PREFETCH = P <= 6;
};

// The lower operands of shifts 2t and 2t+1 of one stage are the same lower-
// block sum T(2b+1, ., t) at columns c + t and c + t + 1 (ceil(s/2) in the
// recursion above).  A lane reads only the first from LDS and takes the second
// from lane + 1 of its wave with a DPP wave shift (lane 63 receives 0), which
// halves the LDS reads of a stage; the first kLaneStages stages need no LDS
// at all.  So that the lanes a column reads are in its own wave, consecutive
// waves overlap by K = 2^kLaneStages - 1 columns: lanes 64 - K .. 63 of wave q
// hold the columns of lanes 0 .. K - 1 of wave q + 1, only the latter copies
// are kept (the duplicates write their operands to a spare LDS column that no
// lane reads, and store nothing), and the last wave's top K lanes are halo.
__device__ __forceinline__ int32_t from_next_lane(int32_t x) {
    return __builtin_amdgcn_mov_dpp(x, 0x130 /* wave_shl:1 */, 0xf, 0xf, true);
}

// One stage of the recursion on the column held in v, in place: the operands
// of the lower half-blocks go through LDS, and outputs (2t, 2t+1) overwrite
// slots that no later t of the same stage still reads (t runs downwards).
// `col` is the thread's LDS column for reads, `wcol` the one it writes.
template <int N, int J, int RW>
__device__ __forceinline__ void fht_stage(int32_t (&v)[N], int32_t* lds, int col, int wcol) {
    constexpr int half = 1 << (J - 1);
    constexpr int blocks = N >> J;
    // The lane's LDS byte address, made opaque to the optimiser so that per-row
    // addresses are formed next to their use instead of being hoisted out of
    // the loop into one register per row.
    unsigned int lane_addr = (unsigned int)(col * RW) * 4u;
    __syncthreads();  // the previous stage's LDS reads are complete
#pragma unroll
    for (int b = 0; b < blocks; ++b)
#pragma unroll
        for (int t = 0; t < half; ++t) lds[wcol * RW + b * half + t] = v[b * 2 * half + half + t];
    __syncthreads();
    // Groups of at most 16 operand pairs, with scheduling barriers between
    // them, so the compiler cannot hoist every LDS read of the stage at once
    // (that would need 2n live registers).
    constexpr int G = half < 16 ? half : 16;
#pragma unroll
    for (int b = 0; b < blocks; ++b) {
#pragma unroll
        for (int g = half / G - 1; g >= 0; --g) {
            asm volatile("" : "+v"(lane_addr));
            const char* lbase = reinterpret_cast<const char*>(lds) + lane_addr;
#pragma unroll
            for (int t = g * G + G - 1; t >= g * G; --t) {
                const int32_t a = v[b * 2 * half + t];
                const int32_t x =
                    *reinterpret_cast<const int32_t*>(lbase + (t * RW + b * half + t) * 4);
                v[b * 2 * half + 2 * t + 1] = a + from_next_lane(x);
                v[b * 2 * half + 2 * t] = a + x;
            }
            __builtin_amdgcn_sched_barrier(0);
        }
    }
}

// The same stage with no scheduling constraints: the compiler may issue all
// LDS reads of the stage together (more registers, more memory parallelism).
// In place, t downwards as above: a second array for the outputs made the
// compiler spill registers at n = 128 (their scratch traffic showed up as
// extra HBM writes).
template <int N, int J, int RW>
__device__ __forceinline__ void fht_stage_free(int32_t (&v)[N], int32_t* lds, int col, int wcol) {
    constexpr int half = 1 << (J - 1);
    constexpr int blocks = N >> J;
    __syncthreads();
#pragma unroll
    for (int b = 0; b < blocks; ++b)
#pragma unroll
        for (int t = 0; t < half; ++t) lds[wcol * RW + b * half + t] = v[b * 2 * half + half + t];
    __syncthreads();
#pragma unroll
    for (int b = 0; b < blocks; ++b) {
#pragma unroll
        for (int t = half - 1; t >= 0; --t) {
            const int32_t a = v[b * 2 * half + t];
            const int32_t x = lds[(col + t) * RW + b * half + t];
            v[b * 2 * half + 2 * t + 1] = a + from_next_lane(x);
            v[b * 2 * half + 2 * t] = a + x;
        }
    }
    // The stage's sums are final here.  Integer adds reassociate freely, and
    // without this the compiler carried partial sums of several stages at once
    // (at n = 128 with 16-bit pixels: 256 VGPRs and 6 spilled; pinned: 188).
#pragma unroll
    for (int q = 0; q < N; ++q) asm volatile("" : "+v"(v[q]));
}

template <int N, int J, int P, int RW, bool GROUPED>
__device__ __forceinline__ void fht_stages(int32_t (&v)[N], int32_t* lds, int col, int wcol) {
    if constexpr (J <= P && J <= kLaneStages) {
        // Shifts 2t and 2t+1 add the lower block's shift t at columns c + t and
        // c + t + 1, i.e. lanes + t and + t + 1: moved by wave shifts, with no
        // LDS exchange and no barrier (the next LDS stage opens with one).
        constexpr int half = 1 << (J - 1);
#pragma unroll
        for (int b = 0; b < (N >> J); ++b) {
            int32_t o[2 * half];
#pragma unroll
            for (int t = 0; t < half; ++t) {
                const int32_t a = v[b * 2 * half + t];
                int32_t x = v[b * 2 * half + half + t];
#pragma unroll
                for (int q = 0; q < t; ++q) x = from_next_lane(x);
                o[2 * t] = a + x;
                o[2 * t + 1] = a + from_next_lane(x);
            }
#pragma unroll
            for (int q = 0; q < 2 * half; ++q) v[b * 2 * half + q] = o[q];
        }
#pragma unroll
        for (int q = 0; q < N; ++q) asm volatile("" : "+v"(v[q]));  // as after an LDS stage
        fht_stages<N, J + 1, P, RW, GROUPED>(v, lds, col, wcol);
    } else if constexpr (J <= P) {
        if constexpr (GROUPED)
            fht_stage<N, J, RW>(v, lds, col, wcol);
        else
            fht_stage_free<N, J, RW>(v, lds, col, wcol);
        fht_stages<N, J + 1, P, RW, GROUPED>(v, lds, col, wcol);
    }
}

// One run of the register kernel for one image: its row blocks of 2^P rows,
// both directions, split into column tiles.  A launch takes a pack of runs
// (several images of the same band height) and numbers their work items
// consecutively from item0.
struct FhtJob {
    const void* img;  // first row of row block 0
    int32_t* out;     // tables [blocks][2n-1][W], or sub-block scratch
    uint16_t* out16;  // narrow tables: bands 0 .. narrow-1 as [narrow][2n-1][W] uint16
    int w, W;         // image width, table width (w + band height)
    int T, tiles;     // columns produced per tile, tiles per row block
    int item0;        // first work item of this run in the launch
    int to_table;     // 1: band tables; 0: c-space sub-block scratch
    int narrow;       // bands stored as uint16 (the rest, from band `narrow` on, go to out)
    int sub16;        // scratch as uint16 (8-bit pixels: a 128-row sum is at most 32640)
};

constexpr int kPack = 256;  // runs per launch (kernel arguments of up to 32 KB)
constexpr int kXcds = 8;   // accelerator dies of the MI355X, each with its own L2

// CAP runs per launch: 1 for a single image (small kernel arguments), kPack for batches.
template <int CAP>
struct FhtPack {
    FhtJob job[CAP];
    int count;  // runs in this pack
    int total;  // work items in this launch
};

// The run a work item belongs to (uniform across the workgroup).
template <int CAP>
__device__ __forceinline__ int fht_find_job(const FhtPack<CAP>& pk, int item) {
    // the last job whose first item is <= item (item0 ascends): binary search
    int lo = 0;
    if constexpr (CAP > 1) {
        int hi = pk.count - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (pk.job[mid].item0 <= item)
                lo = mid;
            else
                hi = mid - 1;
        }
    }
    return lo;
}

struct FhtItem {
    int blk, dir, c, ximg;
    bool inside;
};

// Items of a row block alternate between the two directions, right-leaning
// tiles left to right and left-leaning tiles (whose c-space runs right to
// left in the image) in reverse, so consecutive items read overlapping image
// columns: right tile t and left tile tiles-1-t share most of their pixels.
template <int NDIR>
__device__ __forceinline__ FhtItem fht_decode(const FhtJob& J, int local, int col) {
    FhtItem it;
    const int per_blk = NDIR * J.tiles;
    it.blk = local / per_blk;
    const int u = local - it.blk * per_blk;
    it.dir = NDIR == 2 ? (u & 1) : 0;
    const int t = NDIR == 2 ? (u >> 1) : u;
    const int tile = it.dir ? J.tiles - 1 - t : t;
    it.c = tile * J.T + col;
    const int cm = it.c % J.W;
    it.ximg = it.dir == 0 ? cm : (J.W - 1 - cm);
    it.inside = it.ximg < J.w;
    return it;
}

// Pixels of one c-space column, two rows per 32-bit register.  The row block
// base is uniform (scalar registers), rows are scalar offsets, and the column
// is one 32-bit lane offset shared by every row.
template <int N, int NPK, int NDIR, typename PixT>
__device__ __forceinline__ void fetch_column(const FhtJob& J, int local, int col,
                                             uint32_t (&pk)[NPK]) {
    const FhtItem it = fht_decode<NDIR>(J, local, col);
    const PixT* img = static_cast<const PixT*>(J.img);
    const unsigned int row_bytes = (unsigned int)J.w * sizeof(PixT);
    const __amdgpu_buffer_rsrc_t r =
        make_rsrc(img + (size_t)it.blk * N * (size_t)J.w, (unsigned int)N * row_bytes);
    const unsigned int voff = (it.inside ? (unsigned int)it.ximg : 0u) * sizeof(PixT);
    // Row offsets advance in one scalar register that the optimiser cannot
    // precompute: it had hoisted every row's offset (of loads and of stores)
    // out of the item loop into scalar registers, and spilled them.
    unsigned int so = 0;
#pragma unroll
    for (int q = 0; q < NPK; ++q) {
        const uint32_t lo = buffer_pixel<PixT>(r, voff, so);
        uint32_t hi = 0u;
        if constexpr (N > 1) hi = buffer_pixel<PixT>(r, voff, so + row_bytes);
        pk[q] = it.inside ? (lo | (hi << 16)) : 0u;
        so += 2 * row_bytes;
        asm volatile("" : "+s"(so));
    }
}

// Same pixels straight into the running-sum registers (no prefetch).
template <int N, int NDIR, typename PixT>
__device__ __forceinline__ void fetch_column_direct(const FhtJob& J, int local, int col,
                                                    int32_t (&v)[N]) {
    const FhtItem it = fht_decode<NDIR>(J, local, col);
    const PixT* img = static_cast<const PixT*>(J.img);
    const unsigned int row_bytes = (unsigned int)J.w * sizeof(PixT);
    const __amdgpu_buffer_rsrc_t r =
        make_rsrc(img + (size_t)it.blk * N * (size_t)J.w, (unsigned int)N * row_bytes);
    // Lanes past the image read beyond the buffer extent, which returns 0.
    const unsigned int voff = it.inside ? (unsigned int)it.ximg * sizeof(PixT) : 0x80000000u;
    unsigned int so = 0;
#pragma unroll
    for (int y = 0; y < N; ++y) {
        v[y] = (int32_t)buffer_pixel<PixT>(r, voff, so);
        so += row_bytes;
        asm volatile("" : "+s"(so));
    }
}

// Output modes of a run:
//   to_table: tables[blk][n-1 +- s][x] of a band of n = 2^P rows (d = 0 only from dir 0);
//   else:     scratch[(blk*2 + dir)*2^P + s][c] in c-space (pass 1 of tall bands).
template <int P>
__device__ __forceinline__ void fht_store(const FhtJob& J, int local, int col,
                                          const int32_t (&v)[1 << P]) {
    using C = RegCfg<P>;
    constexpr int N = C::N;
    const FhtItem it = fht_decode<C::NDIR>(J, local, col);
    const int W = J.W;
    if (col >= J.T || it.c >= W) return;
    const unsigned int row_bytes = (unsigned int)W * 4u;
    if (J.to_table && it.blk < J.narrow) {
        // 16-bit table of a band whose line sums stay below 2^16
        constexpr int D = 2 * N - 1;
        const unsigned int row16 = (unsigned int)W * 2u;
        const unsigned int voff = (unsigned int)(it.dir == 0 ? it.c : (W - 1 - it.c)) * 2u;
        const __amdgpu_buffer_rsrc_t r =
            make_rsrc(J.out16 + (size_t)it.blk * D * (size_t)W, (unsigned int)D * row16);
        if (it.dir == 0) {
            unsigned int so = (unsigned int)(N - 1) * row16;
#pragma unroll
            for (int s = 0; s < N; ++s) {
                __builtin_amdgcn_raw_buffer_store_b16((unsigned short)v[s], r, (int)voff, (int)so, 0);
                so += row16;
                asm volatile("" : "+s"(so));
            }
        } else {
            unsigned int so = (unsigned int)(N - 2) * row16;
#pragma unroll
            for (int s = 1; s < N; ++s) {
                __builtin_amdgcn_raw_buffer_store_b16((unsigned short)v[s], r, (int)voff, (int)so, 0);
                so -= row16;
                asm volatile("" : "+s"(so));
            }
        }
    } else if (J.to_table) {
        constexpr int D = 2 * N - 1;
        const unsigned int voff = (unsigned int)(it.dir == 0 ? it.c : (W - 1 - it.c)) * 4u;
        const __amdgpu_buffer_rsrc_t r = make_rsrc(
            J.out + (size_t)(it.blk - J.narrow) * D * (size_t)W, (unsigned int)D * row_bytes);
        if (it.dir == 0) {
            unsigned int so = (unsigned int)(N - 1) * row_bytes;
#pragma unroll
            for (int s = 0; s < N; ++s) {
                __builtin_amdgcn_raw_buffer_store_b32(v[s], r, (int)voff, (int)so, 0);
                so += row_bytes;
                asm volatile("" : "+s"(so));
            }
        } else {
            unsigned int so = (unsigned int)(N - 2) * row_bytes;
#pragma unroll
            for (int s = 1; s < N; ++s) {
                __builtin_amdgcn_raw_buffer_store_b32(v[s], r, (int)voff, (int)so, 0);
                so -= row_bytes;
                asm volatile("" : "+s"(so));
            }
        }
    } else if (J.sub16) {
        const unsigned int row16 = (unsigned int)W * 2u;
        const __amdgpu_buffer_rsrc_t r = make_rsrc(
            reinterpret_cast<uint16_t*>(J.out) + (size_t)(it.blk * C::NDIR + it.dir) * N * (size_t)W,
            (unsigned int)N * row16);
        const unsigned int voff = (unsigned int)it.c * 2u;
        unsigned int so = 0;
#pragma unroll
        for (int s = 0; s < N; ++s) {
            __builtin_amdgcn_raw_buffer_store_b16((unsigned short)v[s], r, (int)voff, (int)so, 0);
            so += row16;
            asm volatile("" : "+s"(so));
        }
    } else {
        const __amdgpu_buffer_rsrc_t r =
            make_rsrc(J.out + (size_t)(it.blk * C::NDIR + it.dir) * N * (size_t)W,
                      (unsigned int)N * row_bytes);
        const unsigned int voff = (unsigned int)it.c * 4u;
        unsigned int so = 0;
#pragma unroll
        for (int s = 0; s < N; ++s) {
            __builtin_amdgcn_raw_buffer_store_b32(v[s], r, (int)voff, (int)so, 0);
            so += row_bytes;
            asm volatile("" : "+s"(so));
        }
    }
}

// Work item = (run, row block, direction, column tile).  The grid holds as
// many workgroups as the chip keeps resident and loops over the items, so a
// workgroup's table stores drain while it loads and transforms its next item;
// the prefetching variants also fetch the next item's pixels while the
// current one runs its stages.  A tile produces T columns (T <= NC - (n-1));
// the rest of its NC columns are halo.
template <int P, typename PixT, int CAP>
__global__ __launch_bounds__(RegCfg<P>::NT) void fht_reg_kernel(FhtPack<CAP> pk) {
    using C = RegCfg<P>;
    constexpr int N = C::N;
    __shared__ int32_t lds[C::LDS_WORDS];
    const int tid = threadIdx.x;
    const int total = pk.total;
    // The thread's column within the tile (waves overlap by K columns).
    const int col = (tid >> 6) * (64 - C::K) + (tid & 63);
    const bool wr = (tid & 63) < 64 - C::K || (tid >> 6) == C::NT / 64 - 1;  // not a duplicate
    const int wcol = wr ? col : C::SPARE;

    uint32_t pre[C::NPK];
    // Workgroups are spread over the XCDs round-robin (workgroup b on XCD
    // b % 8).  Each XCD is given a contiguous run of items instead, so the
    // tiles that share pixel columns meet in one L2: slot i of the launch
    // (workgroup i % grid, round i / grid) takes item xmap(i), which lies in
    // the run of XCD i % 8 whenever the grid is a multiple of 8 or covers
    // every item in one round.
    auto xmap = [total](int i) {
        const int xcd = i % kXcds, slot = i / kXcds;
        return xcd * (total / kXcds) + min(xcd, total % kXcds) + slot;
    };
    const int grid = (int)gridDim.x;
    int vi = blockIdx.x;
    int item = xmap(vi);
    if constexpr (C::PREFETCH) {
        const int j = fht_find_job(pk, item);
        fetch_column<N, C::NPK, C::NDIR, PixT>(pk.job[j], item - pk.job[j].item0, col, pre);
    }
    while (vi < total) {
        const int j = fht_find_job(pk, item);
        const FhtJob& J = pk.job[j];
        const int local = item - J.item0;
        int32_t v[N];
        if constexpr (C::PREFETCH) {
#pragma unroll
            for (int q = 0; q < C::NPK; ++q) {
                v[2 * q] = (int32_t)(pre[q] & 0xffffu);
                if (2 * q + 1 < N) v[2 * q + 1] = (int32_t)(pre[q] >> 16);
            }
        } else {
            fetch_column_direct<N, C::NDIR, PixT>(J, local, col, v);
        }
        vi += grid;
        if constexpr (C::PREFETCH) {
            // Unconditional prefetch (the last round re-reads its own item).
            const int nx = vi < total ? xmap(vi) : item;
            const int jn = fht_find_job(pk, nx);
            fetch_column<N, C::NPK, C::NDIR, PixT>(pk.job[jn], nx - pk.job[jn].item0, col, pre);
        }

        if constexpr (sizeof(PixT) == 1 && P >= 2) {
            // Stages 1 .. p-1 never mix the top and bottom halves of the
            // block, and apply the same shifts to both.  With 8-bit pixels a
            // half's sums stay below 2^16 (at most 64 * 255), so row y and row
            // y + n/2 share a register (low and high 16 bits, no carry between
            // them) and those stages run as the recursion of a block of n/2
            // rows on n/2 registers: half the LDS exchange and half the adds.
            constexpr int H = N / 2;
            int32_t pk[H];
#pragma unroll
            for (int y = 0; y < H; ++y) pk[y] = v[y] | (v[y + H] << 16);
            fht_stages<H, 1, P - 1, C::RW, C::PREFETCH>(pk, lds, col, wcol);
#pragma unroll
            for (int t = 0; t < H; ++t) {
                v[t] = pk[t] & 0xffff;
                v[t + H] = (int32_t)((uint32_t)pk[t] >> 16);
            }
            fht_stages<N, P, P, C::RW, C::PREFETCH>(v, lds, col, wcol);  // the last stage, unpacked
        } else {
            fht_stages<N, 1, P, C::RW, C::PREFETCH>(v, lds, col, wcol);
        }
        if (wr) fht_store<P>(J, local, col, v);
        if (vi < total) item = xmap(vi);
    }
}

// Pass 2 for bands of n = 2^p > 2^7 rows: the band is M = n/128 sub-blocks whose
// FHTs (fine shift sf = s >> (p-7)) sit in `sub`; the line of shift s starts in
// sub-block m at c + D_s(m*128), so T(c, s) = sum_m sub[m][sf][(c + D_s(128 m)) mod W].
// A workgroup covers 256 columns of one (band, direction) for kShiftGroup
// consecutive shifts; the offsets D_s(128 m) are uniform (scalar) per shift.
struct CombineJob {
    const void* sub;   // [sub-blocks][2][128][W] int32, or uint16 for 8-bit pixels (sub16)
    int32_t* tables;   // wide bands (from band `narrow` on), [.][2n-1][W] int32
    uint16_t* tab16;   // narrow bands 0 .. narrow-1, [.][2n-1][W] uint16
    int p, W, k, tiles_x;
    int item0;
    int narrow;
    int sub16;
};

struct CombinePack {
    CombineJob job[kPack];
    int count;
    int total;
};

constexpr int kShiftGroup = 16;

// dyadic_offset(7 + SH, s, m << 7): only the bits of m are set in the row, and
// bit b of m is row bit 7 + b, i.e. j = SH - 1 - b of the closed form.  Every
// shift is a constant, so the offsets cost a handful of scalar operations.
template <int SH>
__device__ __forceinline__ int sub_block_offset(int s, int m) {
    int off = 0;
#pragma unroll
    for (int b = 0; b < SH; ++b)
        if ((m >> b) & 1) off += (s >> (SH - b)) + ((s >> (SH - 1 - b)) & 1);
    return off;
}

// SH = p - 7, M = 2^SH sub-blocks per band; SubT: the scratch's cell type.
template <int SH, typename SubT>
__global__ __launch_bounds__(256) void fht_combine_kernel(CombinePack pk) {
    constexpr int M = 1 << SH;
    const int item = blockIdx.x;
    int j = 0;
    for (int hi = pk.count - 1; j < hi;) {  // last job with item0 <= item
        const int mid = (j + hi + 1) >> 1;
        if (pk.job[mid].item0 <= item)
            j = mid;
        else
            hi = mid - 1;
    }
    const CombineJob& J = pk.job[j];
    const int p = J.p;
    const int n = 1 << p;
    const int D = 2 * n - 1;
    const int W = J.W;
    const int groups = n / kShiftGroup;
    int local = item - J.item0;  // ((band * 2 + dir) * groups + g) * tiles_x + tile
    const int tile = local % J.tiles_x;
    local /= J.tiles_x;
    const int g = local % groups;
    const int bd = local / groups;
    const int dir = bd & 1;
    const int band = bd >> 1;
    const int c = tile * 256 + threadIdx.x;
    if (c >= W) return;
    const size_t row = (size_t)W;
    const SubT* base = static_cast<const SubT*>(J.sub) + (size_t)band * M * 2 * (1 << kRegMaxP) * row;
    const bool n16 = band < J.narrow;
    int32_t* out = J.tables + (size_t)(band - J.narrow) * D * row;
    uint16_t* out16 = J.tab16 + (size_t)band * D * row;
    const int xo = dir == 0 ? c : (W - 1 - c);
    // Every load of the workgroup's shifts first (all in flight together),
    // then the sums and the stores.
    int32_t acc[kShiftGroup];
#pragma unroll
    for (int t = 0; t < kShiftGroup; ++t) {
        const int s = g * kShiftGroup + t;
        const int sf = s >> SH;
        int32_t a = 0;
#pragma unroll
        for (int m = 0; m < M; ++m) {
            int cc = c + sub_block_offset<SH>(s, m);
            cc -= cc >= W ? W : 0;  // offsets are below n < W, so one wrap at most
            a += (int32_t)base[((size_t)(m * 2 + dir) * (1 << kRegMaxP) + sf) * row + cc];
        }
        acc[t] = a;
    }
#pragma unroll
    for (int t = 0; t < kShiftGroup; ++t) {
        const int s = g * kShiftGroup + t;
        if (dir == 1 && s == 0) continue;
        const int r = dir == 0 ? (n - 1 + s) : (n - 1 - s);
        if (n16)
            out16[(size_t)r * row + xo] = (uint16_t)acc[t];
        else
            out[(size_t)r * row + xo] = acc[t];
    }
}

constexpr int kMaxDevices = 64;

int current_device() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
        (void)hipGetLastError();
        return 0;
    }
    return dev;
}

// Compute units of the current device, queried once per device.
int device_cus() {
    static std::atomic<int> cus[kMaxDevices];
    const int dev = current_device();
    int c = cus[dev].load(std::memory_order_relaxed);
    if (c <= 0) {
        if (hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            c <= 0) {
            (void)hipGetLastError();
            c = 256;
        }
        cus[dev].store(c, std::memory_order_relaxed);
    }
    return c;
}

// One register-kernel run to schedule (host side).
struct RegRun {
    const void* img;
    int dtype, p;   // pixel type, log2 of the row-block height the kernel runs
    int w, W, blocks, to_table;
    int32_t* out;
    uint16_t* out16;
    int narrow;
    int grid_mode;  // 0: resident grid; 1: one workgroup per item
    int sub16;
};

template <int P, typename PixT, int CAP>
hipError_t launch_reg_pack(const RegRun* runs, int count, hipStream_t stream) {
    using C = RegCfg<P>;
    // resident workgroups per CU for this instantiation, per device
    static std::atomic<int> occ_of[kMaxDevices];
    const int dev = current_device();
    int occupancy = occ_of[dev].load(std::memory_order_relaxed);
    if (occupancy <= 0) {
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occupancy, fht_reg_kernel<P, PixT, CAP>,
                                                         C::NT, 0) != hipSuccess ||
            occupancy <= 0) {
            (void)hipGetLastError();
            occupancy = 1;
        }
        occ_of[dev].store(occupancy, std::memory_order_relaxed);
    }
    const int Tmax = C::NC - (C::N - 1);
    FhtPack<CAP> pk{};
    long long total = 0;
    for (int q = 0; q < count; ++q) {
        const RegRun& r = runs[q];
        // Tile width: the fewest tiles per row block of at most Tmax columns,
        // spread evenly so every tile does about the same work.
        const int tiles = (r.W + Tmax - 1) / Tmax;
        FhtJob& J = pk.job[q];
        J.img = r.img;
        J.out = r.out;
        J.w = r.w;
        J.W = r.W;
        J.tiles = tiles;
        J.T = (r.W + tiles - 1) / tiles;
        J.item0 = (int)total;
        J.to_table = r.to_table;
        J.out16 = r.out16;
        J.narrow = r.narrow;
        J.sub16 = r.sub16;
        total += (long long)tiles * r.blocks * C::NDIR;
        if (total > 0x7fffffffLL) return hipErrorInvalidConfiguration;
    }
    pk.count = count;
    pk.total = (int)total;
    if (total == 0) return hipSuccess;
    // Resident grid (as many workgroups as the chip keeps, looping over the
    // items) unless the pack asks for one workgroup per item.
    const long long slots = runs[0].grid_mode ? total : (long long)occupancy * device_cus();
    const int grid = (int)(total < slots ? total : slots);
    {
        TimedLaunch tl("fht_reg_kernel", stream);
        hipLaunchKernelGGL((fht_reg_kernel<P, PixT, CAP>), dim3(grid), dim3(C::NT), 0, stream, pk);
    }
    return hipGetLastError();
}

template <typename PixT, int CAP>
hipError_t launch_reg_p(int p, const RegRun* runs, int count, hipStream_t stream) {
    switch (p) {
        case 0: return launch_reg_pack<0, PixT, CAP>(runs, count, stream);
        case 1: return launch_reg_pack<1, PixT, CAP>(runs, count, stream);
        case 2: return launch_reg_pack<2, PixT, CAP>(runs, count, stream);
        case 3: return launch_reg_pack<3, PixT, CAP>(runs, count, stream);
        case 4: return launch_reg_pack<4, PixT, CAP>(runs, count, stream);
        case 5: return launch_reg_pack<5, PixT, CAP>(runs, count, stream);
        case 6: return launch_reg_pack<6, PixT, CAP>(runs, count, stream);
        case 7: return launch_reg_pack<7, PixT, CAP>(runs, count, stream);
        default: return hipErrorInvalidValue;
    }
}

template <typename PixT>
hipError_t launch_reg_any(int p, const RegRun* runs, int count, hipStream_t stream) {
    return count == 1 ? launch_reg_p<PixT, 1>(p, runs, count, stream)
                      : launch_reg_p<PixT, kPack>(p, runs, count, stream);
}

}  // namespace

size_t fht_scratch_bytes(const Geometry& g, int dtype) {
    if (g.p <= kRegMaxP) return 0;
    // [h/128 sub-blocks][2 directions][128 shifts][W]: uint16 for 8-bit pixels
    // (a 128-row line sum is at most 128 * 255), int32 for 16-bit ones
    const size_t cell = dtype == 0 ? sizeof(uint16_t) : sizeof(int32_t);
    return (size_t)(g.h >> kRegMaxP) * 2 * (1u << kRegMaxP) * (size_t)g.W * cell;
}

hipError_t launch_fht_jobs(const FhtJobSpec* jobs, int count, hipStream_t stream) {
    // Register-kernel runs, launched in packs of equal (row-block height, pixel type).
    std::vector<RegRun> runs;
    runs.reserve(count);
    for (int q = 0; q < count; ++q) {
        const FhtJobSpec& J = jobs[q];
        const Geometry& g = J.g;
        RegRun r;
        r.img = J.img;
        r.dtype = J.dtype;
        r.w = g.w;
        r.W = g.W;
        r.out16 = J.tables.narrow ? J.tables.tab16 : nullptr;
        r.narrow = 0;
        r.grid_mode = J.grid_mode;
        r.sub16 = 0;
        if (g.p <= kRegMaxP) {
            r.p = g.p;
            r.blocks = g.k;
            r.to_table = 1;
            r.out = J.tables.wide;
            r.narrow = J.tables.narrow;
        } else {  // tall bands: 128-row sub-blocks first, then the coarse levels
            r.p = kRegMaxP;
            r.blocks = g.h >> kRegMaxP;
            r.to_table = 0;
            r.out = static_cast<int32_t*>(J.scratch);
            r.sub16 = J.dtype == 0;
        }
        runs.push_back(r);
    }
    for (int dtype = 0; dtype < 2; ++dtype) {
        for (int p = 0; p <= kRegMaxP; ++p) {
            for (int gm = 0; gm < 2; ++gm) {
            std::vector<RegRun> group;
            for (const RegRun& r : runs)
                if (r.dtype == dtype && r.p == p && r.grid_mode == gm) group.push_back(r);
            for (size_t q0 = 0; q0 < group.size(); q0 += kPack) {
                const int n = (int)std::min<size_t>(kPack, group.size() - q0);
                hipError_t e = dtype == 0 ? launch_reg_any<uint8_t>(p, group.data() + q0, n, stream)
                                          : launch_reg_any<uint16_t>(p, group.data() + q0, n, stream);
                if (e != hipSuccess) return e;
            }
            }
        }
    }
    // Coarse levels of the tall bands.
    std::vector<CombineJob> comb;
    for (int q = 0; q < count; ++q) {
        const Geometry& g = jobs[q].g;
        if (g.p <= kRegMaxP) continue;
        CombineJob c;
        c.sub = jobs[q].scratch;
        c.sub16 = jobs[q].dtype == 0;
        c.tables = jobs[q].tables.wide;
        c.tab16 = jobs[q].tables.tab16;
        c.narrow = jobs[q].tables.narrow;
        c.p = g.p;
        c.W = g.W;
        c.k = g.k;
        c.tiles_x = (g.W + 255) / 256;
        c.item0 = 0;
        comb.push_back(c);
    }
    for (int sh = 1; sh <= 3; ++sh) {
      for (int s16 = 0; s16 < 2; ++s16) {
        std::vector<CombineJob> group;
        for (const CombineJob& c : comb)
            if (c.p - kRegMaxP == sh && c.sub16 == s16) group.push_back(c);
        for (size_t q0 = 0; q0 < group.size(); q0 += kPack) {
            CombinePack pk{};
            const int n = (int)std::min<size_t>(kPack, group.size() - q0);
            long long total = 0;
            for (int q = 0; q < n; ++q) {
                pk.job[q] = group[q0 + q];
                pk.job[q].item0 = (int)total;
                total += (long long)pk.job[q].tiles_x * ((1LL << pk.job[q].p) / kShiftGroup) * 2 *
                         pk.job[q].k;
                if (total > 0x7fffffffLL) return hipErrorInvalidConfiguration;
            }
            pk.count = n;
            pk.total = (int)total;
            TimedLaunch tl("fht_combine_kernel", stream);
            const dim3 grid((unsigned)total), block(256);
            if (s16) {
                if (sh == 1)
                    hipLaunchKernelGGL((fht_combine_kernel<1, uint16_t>), grid, block, 0, stream, pk);
                else if (sh == 2)
                    hipLaunchKernelGGL((fht_combine_kernel<2, uint16_t>), grid, block, 0, stream, pk);
                else
                    hipLaunchKernelGGL((fht_combine_kernel<3, uint16_t>), grid, block, 0, stream, pk);
            } else {
                if (sh == 1)
                    hipLaunchKernelGGL((fht_combine_kernel<1, int32_t>), grid, block, 0, stream, pk);
                else if (sh == 2)
                    hipLaunchKernelGGL((fht_combine_kernel<2, int32_t>), grid, block, 0, stream, pk);
                else
                    hipLaunchKernelGGL((fht_combine_kernel<3, int32_t>), grid, block, 0, stream, pk);
            }
            hipError_t e = hipGetLastError();
            if (e != hipSuccess) return e;
        }
      }
    }
    return hipSuccess;
}

hipError_t launch_fht(const void* img, int dtype, const Geometry& g, const TableSet& tables,
                      void* scratch, hipStream_t stream, int grid_mode) {
    FhtJobSpec j{img, dtype, g, tables, scratch, grid_mode};
    return launch_fht_jobs(&j, 1, stream);
}

}  // namespace fhtp
