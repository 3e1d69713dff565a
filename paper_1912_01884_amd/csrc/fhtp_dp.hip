// Bend-limited dynamic programme over the band tables (Sections 2.2-2.3), the
// global choice of the best polyline (main problem, steps 2-3) and the
// backtrace of eq. (5).
//
// Values: V_{k-1}(x, d) = H_{k-1}(x, d) when x + d lies in [0, w), else -1, and
// for i = k-2 .. 0
//
//   M_{i+1}(x', d) = max over admissible d' of V_{i+1}(x', d')       (range maximum)
//   A_{i+1}(x', d) = the smallest such d' reaching it                 (back-pointer)
//   V_i(x, d)      = H_i(x, d) + M_{i+1}(x + d, d), or -1 when x + d leaves
//                    [0, w) or M is -1                                 (eqs. (3)-(4))
//
// Layout on gfx950: a thread owns one successor column x' (lanes run along x,
// so every load and store is coalesced) and a chunk of DC consecutive
// displacements d.  It loads V_{i+1}(x', d') for the chunk plus the window
// halo, takes the sliding-window maximum with its argmax in registers (van
// Herk / Gil-Werman: suffix maxima and prefix maxima inside blocks of the
// window length, so three max operations per output whatever the window), and
// then writes V_i(x' - d, d), the diagonal gather of eq. (3), and the
// back-pointer A_{i+1}(x', d).  Cells whose successor column leaves the image
// are never written; readers mask them by the same rule instead.
//
// The last step (i = 0) writes neither V_0 nor A_1: each workgroup reduces its
// cells to a packed key ((V + 1) << 32 | ~(x*D + r)) whose maximum is the best
// score with the smallest (x, d) on ties.  One wave per image then reduces the
// keys and walks the back-pointers (eq. (5)): the first successor comes with
// the best key (the last step records, with each workgroup's key, the argmax
// of that cell's window of V_1, so A_1 is never stored), and later ones are
// read several bands per memory round trip by loading every candidate of the
// next bands speculatively.
//
// A query through a point (Sections 2.2-2.3) pins vertex x_j to one column:
// the step that makes V_j marks every cell of another column infeasible, and
// a pin on x_{k-1} or x_k (cells of V_{k-1} with x or x + d off the point) is
// applied where the table H_{k-1} is read as V_{k-1}.  Every other bend stays
// bounded as usual, so the result is the best polyline through the point.
//
// With the fixed window, two steps share a launch (dp_pair_fixed; three with
// dp_triple_fixed where a tuning rule asks for it): a step
// reads V_{i+1} only in its own successor columns and in its displacement rows
// widened by the bound, so a workgroup computes exactly those cells of V_{i+1}
// from V_{i+2} in LDS and goes on to step i, and V_{i+1} never goes through
// memory.
//
// Every launch takes a pack of images (jobs), so a batch of images of
// different sizes shares one launch per step (or pair of steps) instead of one
// per image and step.  One step per launch: an image with k bands takes part
// in the launches s = 0 .. k-2 of its pack (band i = k-2-s).  Two steps per
// launch: images are aligned at their last step (run_steps_paired).
#include <algorithm>
#include <memory>
#include <type_traits>
#include <vector>

#include "fhtp_internal.h"

namespace fhtp {
namespace {

constexpr int kWaves = 4;      // waves per workgroup, one displacement chunk each
constexpr int kMaxFixedB = 16; // largest bend bound with a register-window kernel
constexpr int kDCGeneric = 8;  // displacements per thread in the scanning kernels
constexpr int kPack = 256;     // images per launch (kernel arguments of up to 32 KB)
constexpr int kXcds = 8;       // accelerator dies of the MI355X, each with its own L2

// Cache policy of the value and back-pointer plane stores: device scope
// (SC1), written through the XCD's L2.  The next launch reads the planes from
// every XCD; written through, they reach memory while the kernel runs instead
// of in the L2 write-back at its end, which sits on the critical path of the
// chain of step launches (about 1.2 us per launch at 4096 x 255 cells).
constexpr int kStoreScope = 16;

// One image in one step launch.
struct DpJob {
    const int32_t* vin;       // V_{i+1} (or the table H_{k-1}), rows d'+n-1
    const void* htab;         // H_i: int32, or uint16 for narrow tables (the kernel's TT)
    int32_t* vout;            // V_i (null on the image's last step)
    void* aout;               // A_{i+1} plane (null on the last step)
    unsigned long long* key;  // last step: one packed key per workgroup, else null
    int32_t* succ;            // last step: per key, the row of that cell's best successor
    const int32_t* win;       // mode-1 windows lo[D], hi[D], or null
    int vin_pitch, h_pitch, v_pitch, a_pitch;
    int n, w;
    int bound;    // mode-0 bound (scanning kernel)
    int full;     // windows cover every displacement
    int items_x;  // workgroups along x
    int items_y;  // workgroups along the displacements
    int item0;    // first workgroup of this image in the launch
    int vin_pin;  // pin on the cells read from vin: 0 none, 1 x' == pin, 2 x' + d' == pin
    int vin_pin_x;
    int out_pin_x;  // V_i cells with x != out_pin_x are infeasible (-1: no pin)
};

// CAP images per launch: 1 for a single image (small kernel arguments, which
// are copied with every launch), kPack for batches.
template <int CAP>
struct DpPack {
    DpJob job[CAP];
    int count;
    int total;  // workgroups in the launch
};

// One image in the walk launch.
struct WalkJob {
    const unsigned long long* key;  // keys of the last step (or of the k = 1 argmax)
    const int32_t* succ;            // with each key, the row of that cell's successor (A_1)
    const void* a_base;             // plane j holds A_{j+2}, j = 0 .. k-3
    size_t a_plane;
    const int32_t* win;
    int32_t* score;
    int32_t* xs;
    int n_keys, a_pitch;
    int n, w, k;
    int bound, full;
    // Bands pair_lo .. pair_top were made two per launch (pair_top 0: none).
    // For i = pair_lo, pair_lo + 2, ... < pair_top, planes i-1 and i together
    // hold one plane of PairLinks<AT> (same row pitch): at the cell
    // (d_i, x_{i+1}), d_{i+1} in the low half and the link d_{i+2} that
    // follows it in the high half, so one load gives both links of a pair.
    int pair_lo, pair_top;
    // Bands 1 .. tri_top were made three per launch (0: none): for i = 1, 4,
    // 7, ..., planes i-1, i and i+1 hold d_{i+1}, d_{i+2} and d_{i+3} at the
    // one index (d_i, x_{i+1}).
    int tri_top;
};

template <int CAP>
struct WalkPack {
    WalkJob job[CAP];
    int count;
};

// Work item of workgroup b of a grid of `total`: workgroup b runs on XCD
// b % 8, and each XCD is given a contiguous run of the items, so that
// neighbouring workgroups share an L2.
__device__ __forceinline__ int xcd_run_item(int b, int total) {
    const int xcd = b % kXcds, slot = b / kXcds;
    return xcd * (total / kXcds) + min(xcd, total % kXcds) + slot;
}

template <int CAP>
__device__ __forceinline__ int dp_find_job(const DpPack<CAP>& pk, int item) {
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

__device__ __forceinline__ unsigned long long pack_key(int val, int x, int r, int D) {
    const unsigned int lin = (unsigned int)x * (unsigned int)D + (unsigned int)r;
    return ((unsigned long long)(unsigned int)(val + 1) << 32) | (unsigned long long)(0xffffffffu - lin);
}

__device__ __forceinline__ unsigned long long wave_max_u64(unsigned long long v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        const unsigned long long o = __shfl_xor(v, off, 64);
        v = o > v ? o : v;
    }
    return v;
}

// Feasible cells (x', d') of V_{i+1}: x' in [xlo, xlo + xlen) and x' + d' in
// [tlo, tlo + tlen).  Without a pin both ranges are [0, w).
struct VMask {
    int xlo, xlen, tlo, tlen;
};

__device__ __forceinline__ VMask vmask(int w, int pin, int pin_x) {
    VMask m{0, w, 0, w};
    if (pin == 1) {
        m.xlo = pin_x;
        m.xlen = 1;
    } else if (pin == 2) {
        m.tlo = pin_x;
        m.tlen = 1;
    }
    return m;
}

// The displacements d' whose cells V_{i+1}(x', d') are feasible form one
// range [dlo, dhi] for a column x' (empty when dhi < dlo): d' in
// [-(n-1), n-1] with x' + d' in [tlo, tlo + tlen), and x' passing the pin.
struct DRange {
    int dlo, dhi;
};

__device__ __forceinline__ DRange drange(int n, int xp, const VMask& mk) {
    DRange r;
    r.dlo = max(-(n - 1), mk.tlo - xp);
    r.dhi = min(n - 1, mk.tlo + mk.tlen - 1 - xp);
    if ((unsigned)(xp - mk.xlo) >= (unsigned)mk.xlen) r.dhi = r.dlo - 1;
    return r;
}

// V_{i+1}(x', d'), or -1 outside the feasible range.  The load is
// unconditional (other lanes read element 0, which always exists) and the
// mask is two compares, no branch, so that every load of a tile is in flight
// at once.
__device__ __forceinline__ int load_v(const int32_t* __restrict__ vin, int pitch, int xp, int dp,
                                      int n, const DRange& dr) {
    const bool ok = (dp >= dr.dlo) & (dp <= dr.dhi);
    const unsigned int off =
        ok ? (unsigned int)(dp + n - 1) * (unsigned int)pitch + (unsigned int)xp : 0u;
    const int v = vin[off];
    return ok ? v : -1;
}

// Admissible successors of displacement d: [lo, hi] in displacement units.
__device__ __forceinline__ void window_of(int n, int full, const int32_t* win, int bound, int d,
                                          int& lo, int& hi) {
    if (full) {
        lo = -(n - 1);
        hi = n - 1;
    } else if (win) {
        lo = win[d + n - 1];
        hi = win[2 * n - 1 + d + n - 1];
    } else {
        lo = max(d - bound, -(n - 1));
        hi = min(d + bound, n - 1);
    }
}

// H_i(x' - d, d) for one output cell, 0 where the cell does not exist
// (unconditional load, as load_v).
template <typename TT>
__device__ __forceinline__ int load_h(const DpJob& a, int xp, int d) {
    const int r = d + a.n - 1;
    const int x = xp - d;
    const bool ok = (unsigned)xp < (unsigned)a.w && (unsigned)r < (unsigned)(2 * a.n - 1) &&
                    (unsigned)x < (unsigned)a.w;
    const unsigned int off = ok ? (unsigned int)r * (unsigned int)a.h_pitch + (unsigned int)x : 0u;
    const int v = (int)static_cast<const TT*>(a.htab)[off];
    return ok ? v : 0;
}

// One table cell through a buffer view, at byte offsets computed with the
// table's element size: int32 tables, or uint16 narrow ones (zero-extended).
template <typename TT>
__device__ __forceinline__ int load_tab(__amdgpu_buffer_rsrc_t r, unsigned int voff,
                                        unsigned int soff) {
    if constexpr (sizeof(TT) == 2)
        return (int)__builtin_amdgcn_raw_buffer_load_b16(r, (int)voff, (int)soff, 0);
    else
        return __builtin_amdgcn_raw_buffer_load_b32(r, (int)voff, (int)soff, 0);
}

// The best cell of a thread on the last step: its packed key and the row
// d'+n-1 of its best successor (the back-pointer A_1 the step does not store).
struct Best {
    unsigned long long key = 0;
    int succ = 0;
};

__device__ __forceinline__ void take_best(Best& b, unsigned long long kk, int succ_row) {
    const bool t = kk > b.key;
    b.key = t ? kk : b.key;
    b.succ = t ? (succ_row < 0 ? 0 : succ_row) : b.succ;
}

// Wave-wide best: the largest key (keys of distinct cells differ) and the
// successor held by the lane that has it.
__device__ __forceinline__ Best wave_best(Best b) {
    const unsigned long long m = wave_max_u64(b.key);
    const unsigned long long hit = __builtin_amdgcn_ballot_w64(b.key == m);
    Best r;
    r.key = m;
    r.succ = __builtin_amdgcn_readlane(b.succ, (int)__builtin_ctzll(hit));
    return r;
}

// Common end of a step workgroup: on the image's last step its best key and
// that cell's successor go to slot `slot` (its workgroup index within the image).
__device__ __forceinline__ void finish(const DpJob& a, Best best, int slot) {
    if (!a.key) return;
    __shared__ unsigned long long part[kWaves];
    __shared__ int part_s[kWaves];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    best = wave_best(best);
    if (lane == 0) {
        part[wave] = best.key;
        part_s[wave] = best.succ;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long m = part[0];
        int ms = part_s[0];
#pragma unroll
        for (int q = 1; q < kWaves; ++q) {
            const bool t = part[q] > m;
            m = t ? part[q] : m;
            ms = t ? part_s[q] : ms;
        }
        a.key[slot] = m;
        a.succ[slot] = ms;
    }
}

// Buffer view of rows [row0, row0 + rows) of a plane (pitch elements of esz
// bytes per row), clamped to the plane's rows [0, D).  row0 is wave-uniform,
// so the descriptor lives in scalar registers and every access is a 32-bit
// offset from it: no 64-bit address arithmetic per load, which would tie
// later address computations to registers of loads still in flight.
struct RowView {
    __amdgpu_buffer_rsrc_t rs;
    int base;  // plane row at byte offset 0
    int end;   // one past the last row covered
};

__device__ __forceinline__ RowView row_view(const void* plane, int pitch, int esz, int row0,
                                            int rows, int D) {
    RowView v;
    v.base = min(max(row0, 0), D - 1);
    v.end = min(row0 + rows, D);
    const int cnt = max(v.end - v.base, 1);
    v.rs = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<char*>(static_cast<const char*>(plane)) + (size_t)v.base * pitch * esz,
        (short)0, cnt * pitch * esz, 0x00020000);
    return v;
}

// The two links of a pair of steps in one element: the low half holds a
// cell's own choice, the high half the link after it.
template <typename AT>
using PairLinks = std::conditional_t<sizeof(AT) == 1, uint16_t, uint32_t>;
template <typename AT>
constexpr int kLinkBits = 8 * (int)sizeof(AT);

// Byte offset of a row inside the view (0 for rows it does not cover, whose
// lanes are masked by an out-of-range lane offset instead).
__device__ __forceinline__ unsigned int row_off(const RowView& v, int row, int pitch, int esz) {
    return (row >= v.base && row < v.end) ? (unsigned int)(row - v.base) * pitch * esz : 0u;
}

constexpr unsigned int kOut = 0x80000000u;  // lane offset past every view: loads 0, stores drop

// One output cell (x' = xp, displacement d) with range maximum m reached at
// row ra, stored through the views of the wave's rows of V_i (ov) and
// A_{i+1} (av).
template <typename AT>
__device__ __forceinline__ void emit(const DpJob& a, const RowView& ov, const RowView& av, int m,
                                     int ra, int hval, int xp, int d, Best& best) {
    const int n = a.n, w = a.w;
    const int D = 2 * n - 1;
    const int r = d + n - 1;
    if (xp >= w || r >= D) return;
    const bool last = a.key != nullptr;
    if (!last) {
        const unsigned int arow = row_off(av, r, a.a_pitch, sizeof(AT));
        const unsigned int aval = (unsigned int)(ra < 0 ? 0 : ra);
        if constexpr (sizeof(AT) == 1)
            __builtin_amdgcn_raw_buffer_store_b8((unsigned char)aval, av.rs, xp, (int)arow,
                                                 kStoreScope);
        else
            __builtin_amdgcn_raw_buffer_store_b16((unsigned short)aval, av.rs, xp * 2, (int)arow,
                                                  kStoreScope);
    }
    const int x = xp - d;
    if (x < 0 || x >= w) return;
    const int val = (m >= 0 && (a.out_pin_x < 0 || x == a.out_pin_x)) ? hval + m : -1;
    if (last) {
        take_best(best, pack_key(val, x, r, D), ra);
    } else {
        __builtin_amdgcn_raw_buffer_store_b32(val, ov.rs, x * 4, (int)row_off(ov, r, a.v_pitch, 4),
                                              kStoreScope);
    }
}

// Sliding maximum of the windows [j, j + 2B] of v, j = 0 .. DC-1, with the
// smallest index reaching it: each window is split at a block start b in
// (j, j + 2B] into the suffix maximum of v[j .. b-1] within its block and the
// prefix maximum of v[b .. j+2B] within the next (van Herk / Gil-Werman).
// When DC <= 2B every window holds both v[DC-1] and v[DC], so the single
// boundary b = DC serves them all; otherwise blocks of 2B start at multiples
// of 2B, and b is the first one above j.  Only the suffixes that start below
// DC and the prefixes that start at a boundary are formed (about two thirds
// of the compares and selects of blocks of the window length over all of v).
// Ties go to the smallest index: suffixes are taken descending on >=,
// prefixes ascending on >, and the suffix (the smaller indices) wins a tie
// between the two.
template <int B, int DC>
__device__ __forceinline__ void window_max(const int (&v)[DC + 2 * B], int (&m)[DC],
                                           int (&ia)[DC]) {
    constexpr int L = 2 * B + 1;
    constexpr int NV = DC + 2 * B;
    if constexpr (DC <= 2 * B) {
        int sv[DC], si[DC];
        sv[DC - 1] = v[DC - 1];
        si[DC - 1] = DC - 1;
#pragma unroll
        for (int q = DC - 2; q >= 0; --q) {
            const bool take = v[q] >= sv[q + 1];
            sv[q] = take ? v[q] : sv[q + 1];
            si[q] = take ? q : si[q + 1];
        }
        int pv = v[DC], pi = DC;
#pragma unroll
        for (int t = DC; t < NV; ++t) {
            if (t > DC && v[t] > pv) {
                pv = v[t];
                pi = t;
            }
            const int j = t - 2 * B;  // the window ending at t
            if (j >= 0 && j < DC) {
                const bool s_wins = sv[j] >= pv;
                m[j] = s_wins ? sv[j] : pv;
                ia[j] = s_wins ? si[j] : pi;
            }
        }
        return;
    } else if constexpr (B >= 1) {
        constexpr int S = 2 * B;
        constexpr int SE = NV < S * ((DC + S - 1) / S) ? NV : S * ((DC + S - 1) / S);
        int sv[SE], si[SE];
#pragma unroll
        for (int q = SE - 1; q >= 0; --q) {
            if (q == SE - 1 || (q + 1) % S == 0) {
                sv[q] = v[q];
                si[q] = q;
            } else {
                const bool take = v[q] >= sv[q + 1];
                sv[q] = take ? v[q] : sv[q + 1];
                si[q] = take ? q : si[q + 1];
            }
        }
        int pv = 0, pi = 0;
#pragma unroll
        for (int t = S; t < NV; ++t) {
            if (t % S == 0) {
                pv = v[t];
                pi = t;
            } else if (v[t] > pv) {
                pv = v[t];
                pi = t;
            }
            const int j = t - 2 * B;  // the window ending at t
            if (j >= 0 && j < DC) {
                const bool s_wins = sv[j] >= pv;
                m[j] = s_wins ? sv[j] : pv;
                ia[j] = s_wins ? si[j] : pi;
            }
        }
        return;
    }
    int sv[NV], si[NV];
#pragma unroll
    for (int q = NV - 1; q >= 0; --q) {
        if (q % L == L - 1 || q == NV - 1) {
            sv[q] = v[q];
            si[q] = q;
        } else {
            const bool take = v[q] >= sv[q + 1];
            sv[q] = take ? v[q] : sv[q + 1];
            si[q] = take ? q : si[q + 1];
        }
    }
    int pv = 0, pi = 0;
#pragma unroll
    for (int q = 0; q < NV; ++q) {
        if (q % L == 0) {
            pv = v[q];
            pi = q;
        } else if (v[q] > pv) {
            pv = v[q];
            pi = q;
        }
        if (q >= 2 * B) {
            const int j = q - 2 * B;  // window [j, q]: suffix of j's block + prefix of q's block
            const bool s_wins = sv[j] >= pv;
            m[j] = s_wins ? sv[j] : pv;
            ia[j] = s_wins ? si[j] : pi;
        }
    }
}

// A wave whose every cell, window row and successor column lies inside the
// image and the planes (and no pin applies) needs no masks: one descriptor
// per plane, one lane offset per access pattern, rows as scalar offsets.
template <int B, int DC>
__device__ __forceinline__ bool wave_is_interior(const DpJob& a, int X0, int r0, int d0) {
    const int D = 2 * a.n - 1, w = a.w;
    return a.vin_pin == 0 && a.out_pin_x < 0 && r0 - B >= 0 && r0 + DC + B <= D &&
           X0 + 64 <= w &&
           X0 + d0 - B >= 0 && X0 + 63 + d0 + DC - 1 + B < w &&  // x' + d' for every window row
           X0 - (d0 + DC - 1) >= 0 && X0 + 63 - d0 < w;          // x = x' - d for every cell
}

template <int B, int DC, typename AT, typename TT>
__device__ __forceinline__ Best fixed_interior(const DpJob& a, int X0, int r0, int d0) {
    constexpr int NV = DC + 2 * B;
    constexpr unsigned int hsz = sizeof(TT);
    const int D = 2 * a.n - 1;
    const int xp = X0 + (int)(threadIdx.x & 63);
    const unsigned int vp = (unsigned int)a.vin_pitch * 4u;
    const unsigned int hp = (unsigned int)a.h_pitch * hsz;
    const __amdgpu_buffer_rsrc_t vr = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<int32_t*>(a.vin) + (size_t)(r0 - B) * a.vin_pitch, (short)0, (int)(NV * vp),
        0x00020000);
    const __amdgpu_buffer_rsrc_t hr = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<TT*>(static_cast<const TT*>(a.htab)) + (size_t)r0 * a.h_pitch, (short)0,
        (int)(DC * hp), 0x00020000);
    // cell j sits at column x' - d0 - j: one lane offset for the row group,
    // the column step as a constant
    const unsigned int diag = (unsigned int)(xp - d0 - (DC - 1)) * hsz;
    int hv[DC], v[NV];
#pragma unroll
    for (int j = 0; j < DC; ++j)
        hv[j] = load_tab<TT>(hr, diag + (DC - 1 - j) * hsz, j * hp);
#pragma unroll
    for (int j = 0; j < NV; ++j)
        v[j] = __builtin_amdgcn_raw_buffer_load_b32(vr, xp * 4, (int)(j * vp), 0);
    __builtin_amdgcn_sched_barrier(0);
    int m[DC], ia[DC];
    window_max<B, DC>(v, m, ia);
    Best best;
    if (a.key) {
#pragma unroll
        for (int j = 0; j < DC; ++j) {
            const int val = m[j] >= 0 ? hv[j] + m[j] : -1;
            take_best(best, pack_key(val, xp - d0 - j, r0 + j, D), r0 - B + ia[j]);
        }
        return best;
    }
    const unsigned int op = (unsigned int)a.v_pitch * 4u;
    const unsigned int ap = (unsigned int)a.a_pitch * sizeof(AT);
    // the V_i cells lie on the same diagonal as the table cells, at 4 bytes a cell
    const unsigned int vdiag = (unsigned int)(xp - d0 - (DC - 1)) * 4u;
    const __amdgpu_buffer_rsrc_t orr = __builtin_amdgcn_make_buffer_rsrc(
        a.vout + (size_t)r0 * a.v_pitch, (short)0, (int)(DC * op), 0x00020000);
    const __amdgpu_buffer_rsrc_t ar = __builtin_amdgcn_make_buffer_rsrc(
        static_cast<AT*>(a.aout) + (size_t)r0 * a.a_pitch, (short)0, (int)(DC * ap), 0x00020000);
#pragma unroll
    for (int j = 0; j < DC; ++j) {
        const int val = m[j] >= 0 ? hv[j] + m[j] : -1;
        const unsigned int row = (unsigned int)(r0 - B + ia[j]);  // d' + n - 1 of the maximum
        if constexpr (sizeof(AT) == 1)
            __builtin_amdgcn_raw_buffer_store_b8((unsigned char)row, ar, xp, (int)(j * ap), kStoreScope);
        else
            __builtin_amdgcn_raw_buffer_store_b16((unsigned short)row, ar, xp * 2, (int)(j * ap), kStoreScope);
        __builtin_amdgcn_raw_buffer_store_b32(val, orr, (int)(vdiag + (DC - 1 - j) * 4),
                                              (int)(j * op), kStoreScope);
    }
    return best;
}

// One wave of a mode-0 step with the window [d - B, d + B] fixed at compile
// time, anywhere in the planes (cells outside the image or the planes,
// pinned columns).  All loads first (the window column of V_{i+1} and the H_i
// cells), then the sliding maximum, then the cells.  A thread's V loads are
// consecutive rows of one column, so the valid ones form a range of the row
// index; H loads are not masked (a cell outside the image only yields a value
// that is never used, and offsets outside a view read 0); stores are masked
// by ranges and every variable offset part sits in the lane offset, which the
// hardware checks against the view's extent.
template <int B, int DC, typename AT, typename TT>
__device__ __forceinline__ Best fixed_general(const DpJob& a, int X0, int r0, int d0) {
    constexpr int NV = DC + 2 * B;
    constexpr int esz = (int)sizeof(AT);
    const int n = a.n, w = a.w;
    const int D = 2 * n - 1;
    const int xp = X0 + (int)(threadIdx.x & 63);
    const bool col_ok = xp < w;

    // H_i(x' - d, d), d = d0 + j: rows r0 + j, column x' - d.
    constexpr unsigned int hsz = sizeof(TT);
    const RowView hview = row_view(a.htab, a.h_pitch, (int)hsz, r0, DC, D);
    const unsigned int hp = (unsigned int)a.h_pitch * hsz;
    const unsigned int hb = (unsigned int)(r0 - hview.base) * hp + (unsigned int)(xp - d0) * hsz;
    int hv[DC];
#pragma unroll
    for (int j = 0; j < DC; ++j) hv[j] = load_tab<TT>(hview.rs, hb + j * (hp - hsz), 0);
    // V_{i+1}(x', d'), d' = d0 - B + q: rows r0 - B + q, column x'; a cell when
    // x' passes the pin, the row lies in [0, D) and x' + d' in [tlo, tlo + tlen).
    const VMask mk = vmask(w, a.vin_pin, a.vin_pin_x);
    const bool xin = (unsigned)(xp - mk.xlo) < (unsigned)mk.xlen;
    const int rlo = r0 - B;
    const int qlo = max(-rlo, mk.tlo - xp - rlo + (n - 1));
    const int qhi = xin ? min(D - rlo, mk.tlo + mk.tlen - xp - rlo + (n - 1)) : qlo;
    const RowView vview = row_view(a.vin, a.vin_pitch, 4, rlo, NV, D);
    const unsigned int vp = (unsigned int)a.vin_pitch * 4u;
    const unsigned int vb = (unsigned int)(rlo - vview.base) * vp + (unsigned int)xp * 4u;
    int v[NV];
#pragma unroll
    for (int q = 0; q < NV; ++q) {
        const bool ok = q >= qlo && q < qhi;
        const int t = __builtin_amdgcn_raw_buffer_load_b32(vview.rs, (int)(ok ? vb + q * vp : kOut),
                                                           0, 0);
        v[q] = ok ? t : -1;
    }
    __builtin_amdgcn_sched_barrier(0);
    int m[DC], ia[DC];
    window_max<B, DC>(v, m, ia);

    // cell j: row r0 + j < D; V_i(x, d) at x = x' - d0 - j in [0, w)
    const int jn = col_ok ? min(DC, D - r0) : 0;
    const int xj = xp - d0;  // x of cell j is xj - j
    const bool last = a.key != nullptr;
    Best best;
    if (last) {
#pragma unroll
        for (int j = 0; j < DC; ++j) {
            const int x = xj - j;
            const bool live = j < jn && (unsigned)x < (unsigned)w;
            const int val = (m[j] >= 0 && (a.out_pin_x < 0 || x == a.out_pin_x)) ? hv[j] + m[j] : -1;
            take_best(best, live ? pack_key(val, x, r0 + j, D) : 0ull, rlo + ia[j]);
        }
        return best;
    }
    const RowView aview = row_view(a.aout, a.a_pitch, esz, r0, DC, D);
    const RowView oview = row_view(a.vout, a.v_pitch, 4, r0, DC, D);
    const unsigned int ap = (unsigned int)a.a_pitch * (unsigned int)esz;
    const unsigned int op = (unsigned int)a.v_pitch * 4u;
    const unsigned int ab = (unsigned int)(r0 - aview.base) * ap + (unsigned int)xp * (unsigned int)esz;
    const unsigned int ob = (unsigned int)(r0 - oview.base) * op + (unsigned int)xj * 4u;
#pragma unroll
    for (int j = 0; j < DC; ++j) {
        const int x = xj - j;
        const bool cell = j < jn;
        const bool live = cell && (unsigned)x < (unsigned)w;
        const int val = (m[j] >= 0 && (a.out_pin_x < 0 || x == a.out_pin_x)) ? hv[j] + m[j] : -1;
        const int ra = rlo + ia[j];  // row of the maximum's d'
        const unsigned int av = (unsigned int)(ra < 0 ? 0 : ra);
        const unsigned int aoff = cell ? ab + j * ap : kOut;
        if constexpr (sizeof(AT) == 1)
            __builtin_amdgcn_raw_buffer_store_b8((unsigned char)av, aview.rs, (int)aoff, 0, kStoreScope);
        else
            __builtin_amdgcn_raw_buffer_store_b16((unsigned short)av, aview.rs, (int)aoff, 0, kStoreScope);
        __builtin_amdgcn_raw_buffer_store_b32(val, oview.rs, (int)(live ? ob + j * (op - 4u) : kOut), 0,
                                              kStoreScope);
    }
    return best;
}

template <int B, int DC, typename AT, typename TT>
__device__ __forceinline__ Best fixed_item(const DpJob& a, int bx, int by) {
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int X0 = bx * 64;
    const int r0 = (by * kWaves + wave) * DC;  // table row of this wave's first displacement
    const int d0 = r0 - (a.n - 1);
    if (wave_is_interior<B, DC>(a, X0, r0, d0))
        return fixed_interior<B, DC, AT, TT>(a, X0, r0, d0);
    return fixed_general<B, DC, AT, TT>(a, X0, r0, d0);
}

// Step with the mode-0 window fixed at compile time.  TT: the table's
// element type (int32, or uint16 for narrow tables).
template <int B, int DC, typename AT, int CAP, typename TT>
__global__ __launch_bounds__(64 * kWaves) void dp_step_fixed(DpPack<CAP> pk) {
    // items of an image run down the displacement groups of one column tile
    // before the next tile, so the window rows shared by vertical neighbours
    // meet in one L2
    const int it = xcd_run_item((int)blockIdx.x, (int)gridDim.x);
    const int j = dp_find_job(pk, it);
    const DpJob& a = pk.job[j];
    const int local = it - a.item0;
    const int bx = local / a.items_y, by = local - bx * a.items_y;
    const Best best = fixed_item<B, DC, AT, TT>(a, bx, by);
    finish(a, best, local);
}

// ---- two steps per launch (fixed mode-0 window) -------------------------------
//
// A step reads V_{i+1} only in the successor columns it owns and in the rows
// of its displacements widened by B on either side, so a workgroup can make
// those cells of V_{i+1} itself from V_{i+2} and go straight on to step i:
//
//   phase 1: V_{i+1}(x', d') for x' in its 64 columns and d' in its rows
//            widened by B, into LDS, as the step for band i+1 computes them
//            (successor column x'' = x' + d', window of V_{i+2} in that
//            column), each with the row of its own window maximum;
//   phase 2: step i from LDS, writing V_i, A_{i+1}, and in the A_{i+2} plane,
//            at the same cell of step i, the link after next: the choice of
//            band i+1 for the V_{i+1} cell that band i chose.  The walk reads
//            both links of a pair at one index.
//
// V_{i+1} then never goes through memory and the chain of dependent launches
// is half as long.  The cells of the widened rows are recomputed by the
// neighbouring workgroups (2B rows on top of 32).  Phase 1 runs in strips of
// kStrip rows: a strip's cells lie in 64 + kStrip - 1 successor columns, one
// thread each.
constexpr int kPairWaves = 4;                    // waves per workgroup
constexpr int kPairDC = 8;                       // phase 2: displacements per thread
constexpr int kPairRows = kPairWaves * kPairDC;  // displacements of step i per workgroup
constexpr int kStrip = 16;                       // phase 1: displacements per thread

struct DpPairJob {
    const int32_t* vin;  // V_{i+2} (or the table H_{k-1}), rows d''+n-1
    const void* h1;      // H_{i+1} (int32, or uint16 for narrow tables: the kernel's TT)
    const void* h0;      // H_i
    int32_t* vout;       // V_i
    // At each cell of step i, PairLinks<AT>: its own choice (row of A_{i+1})
    // and the link after next (the choice of the chosen cell of step i+1);
    // the plane spans what two planes of AT would
    void* a;
    int vin_pitch, h_pitch, v_pitch, a_pitch;
    int n, w, items_x, items_y;
    int item0;  // first workgroup of this image in the launch
    // Through-point pin: on the cells read from vin (the table H_{k-1} read as
    // V_{k-1}: 0 none, 1 x'' == pin, 2 x'' + d'' == pin), and on the cells of
    // V_{i+1} (pin1_x) and V_i (pin0_x) made here (-1: none).
    int vin_pin, vin_pin_x;
    int pin1_x, pin0_x;
};

// CAP images per launch, as DpPack.
template <int CAP>
struct DpPairPack {
    DpPairJob job[CAP];
    int count;
    int stripe;  // column tiles per stripe of the item order (tuned; 16 by default)
};

// Masks: a thread's loads of V_{i+2} are consecutive rows of one column, so
// the valid ones form a range of the row index; table loads are not masked
// at all (a cell outside the image only yields a value that is never used,
// and offsets outside a view read 0); stores are masked by ranges of the
// row index and write nothing outside their rows.  All variable parts of an
// offset go to the lane offset, which is what the hardware checks against
// the view's extent.
// PIN: the through-point masks (a separate instantiation, so that unpinned
// launches carry none of their instructions or registers).
template <int B, typename AT, int CAP, bool PIN, typename TT>
__global__ __launch_bounds__(64 * kPairWaves) void dp_pair_fixed(DpPairPack<CAP> pk) {
    constexpr int RM = kPairRows + 2 * B;  // rows of V_{i+1} the workgroup needs
    constexpr int NS = (RM + kStrip - 1) / kStrip;
    constexpr int SC = 64 + kStrip - 1;    // successor columns of one strip
    constexpr int NV1 = kStrip + 2 * B;
    constexpr int NV2 = kPairDC + 2 * B;
    constexpr int LP = kStrip - 1;         // padding on either side of an LDS row
    constexpr int LWP = 64 + 2 * LP;       // strip cells outside the tile land in the padding
    __shared__ int mid[NS * kStrip][LWP];  // V_{i+1}(X0 + c, row m0 + q) at [q][LP + c]
    __shared__ AT nxt[NS * kStrip][LWP];   // row of that cell's window maximum (its choice)

    // Workgroup b runs on XCD b % 8.  Each XCD gets a contiguous run of items
    // instead, an image's items in stripes of pk.stripe column tiles (every
    // row group of a stripe before the next stripe), so that the overlapping
    // reads of neighbouring workgroups (the widened rows, a strip's extra
    // columns, the diagonal shift between row groups) meet in one L2.
    const int it = xcd_run_item((int)blockIdx.x, (int)gridDim.x);
    int jj = 0;  // the last image whose first item is <= it (item0 ascends)
    if constexpr (CAP > 1) {
        int hi = pk.count - 1;
        while (jj < hi) {
            const int md = (jj + hi + 1) >> 1;
            if (pk.job[md].item0 <= it)
                jj = md;
            else
                hi = md - 1;
        }
    }
    const DpPairJob& a = pk.job[jj];
    const int n = a.n, w = a.w;
    const int D = 2 * n - 1;
    int bx, by;
    {
        const int local = CAP > 1 ? it - a.item0 : it;  // one image: item0 is 0
        const int stripe = pk.stripe;
        const int per_stripe = stripe * a.items_y;
        const int st = local / per_stripe, loc = local - st * per_stripe;
        const int sw = min(stripe, a.items_x - st * stripe);
        by = loc / sw;
        bx = st * stripe + (loc - by * sw);
    }
    const int X0 = bx * 64;
    const int r0 = by * kPairRows;  // table row of the first displacement of step i
    const int m0 = r0 - B;          // table row of mid[0]
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    constexpr unsigned int hsz = sizeof(TT);
    const unsigned int hp = (unsigned int)a.h_pitch * hsz;

    // Phase 2's H_i(x' - d, d), issued first so that the loads overlap phase 1.
    const int xp = X0 + lane;
    const bool col_ok = xp < w;
    const int r2 = r0 + wave * kPairDC;
    const int d2 = r2 - (n - 1);
    const RowView h0v = row_view(a.h0, a.h_pitch, (int)hsz, r2, kPairDC, D);
    const unsigned int h0b = (unsigned int)(r2 - h0v.base) * hp + (unsigned int)(xp - d2) * hsz;
    int hv0[kPairDC];
#pragma unroll
    for (int j = 0; j < kPairDC; ++j) hv0[j] = load_tab<TT>(h0v.rs, h0b + j * (hp - hsz), 0);

    // Phase 1.  Views: V_{i+2} rows [m0 - B, m0 + NS*kStrip + B), H_{i+1} rows
    // [m0, m0 + RM), each clipped to [0, D).
    const RowView vv = row_view(a.vin, a.vin_pitch, 4, m0 - B, NS * kStrip + 2 * B, D);
    const RowView h1v = row_view(a.h1, a.h_pitch, (int)hsz, m0, RM, D);
    const unsigned int vp = (unsigned int)a.vin_pitch * 4u;
    for (int t = threadIdx.x; t < NS * SC; t += 64 * kPairWaves) {
        const int s = t / SC, c = t - s * SC;
        const int q0 = s * kStrip;             // mid row of the strip's first displacement
        const int rs = m0 + q0;                // its table row
        const int xs = X0 + rs - (n - 1) + c;  // successor column x''
        const bool xs_ok = (unsigned)xs < (unsigned)w;
        // v[q] = V_{i+2}(x'', row rs - B + q): a cell when the row lies in
        // [0, D), x'' in [xlo, xlo + xlen) and x'' plus its displacement in
        // [tlo, tlo + tlen) (both [0, w) unless vin carries a pin)
        const VMask mk = PIN ? vmask(w, a.vin_pin, a.vin_pin_x) : VMask{0, w, 0, w};
        const int rlo = rs - B;
        const int qlo = max(-rlo, mk.tlo + (n - 1) - xs - rlo);
        const int qhi = (unsigned)(xs - mk.xlo) < (unsigned)mk.xlen
                            ? min(D - rlo, mk.tlo + mk.tlen + (n - 1) - xs - rlo)
                            : qlo;
        // cell j exists when its row lies in [0, D), x' = X0 + c - j < w and
        // x'' lies in [0, w); it is in the tile when 0 <= c - j < 64
        const int jlo = max(-rs, X0 + c - w + 1);
        const int jhi = xs_ok ? D - rs : jlo;
        const unsigned int vb = (unsigned int)(rlo - vv.base) * vp + (unsigned int)xs * 4u;
        const unsigned int hb = (unsigned int)(rs - h1v.base) * hp + (unsigned int)(X0 + c) * hsz;
        int* lrow = &mid[q0][LP + c];
        AT* nrow = &nxt[q0][LP + c];
        // A wave whose every load and cell is valid takes the unmasked copy.
        const bool inner = qlo <= 0 && qhi >= NV1 && jlo <= 0 && jhi >= kStrip && (!PIN || a.pin1_x < 0);
        auto strip = [&](auto inner_tag) {
            constexpr bool INNER = decltype(inner_tag)::value;
            int v[NV1];
#pragma unroll
            for (int q = 0; q < NV1; ++q) {
                if constexpr (INNER) {
                    v[q] = __builtin_amdgcn_raw_buffer_load_b32(vv.rs, (int)(vb + q * vp), 0, 0);
                } else {
                    const bool ok = q >= qlo && q < qhi;
                    const int tv = __builtin_amdgcn_raw_buffer_load_b32(
                        vv.rs, (int)(ok ? vb + q * vp : kOut), 0, 0);
                    v[q] = ok ? tv : -1;
                }
            }
            // H_{i+1}(x', d') at x' = X0 + c - j, row rs + j
            int hv[kStrip];
#pragma unroll
            for (int j = 0; j < kStrip; ++j)
                hv[j] = load_tab<TT>(h1v.rs, hb + j * (hp - hsz), 0);
            __builtin_amdgcn_sched_barrier(0);
            int m[kStrip], ia[kStrip];
            window_max<B, kStrip>(v, m, ia);
#pragma unroll
            for (int j = 0; j < kStrip; ++j) {
                const bool live =
                    INNER || (j >= jlo && j < jhi && (!PIN || a.pin1_x < 0 || X0 + c - j == a.pin1_x));
                const int val = live && m[j] >= 0 ? hv[j] + m[j] : -1;
                lrow[j * (LWP - 1)] = val;
                const int ra = rs - B + ia[j];  // row of the maximum's d''
                nrow[j * (LWP - 1)] = (AT)(INNER || ra >= 0 ? ra : 0);
            }
        };
        if (__builtin_amdgcn_ballot_w64(!inner) == 0)
            strip(std::true_type{});
        else
            strip(std::false_type{});
    }
    __syncthreads();

    // Phase 2: step i on the LDS copy of V_{i+1}; rows outside [0, D) and
    // cells without a successor column hold -1.
    int v2[NV2];
    const int* lcol = &mid[wave * kPairDC][LP + lane];
#pragma unroll
    for (int q = 0; q < NV2; ++q) v2[q] = lcol[q * LWP];
    int m2[kPairDC], ia2[kPairDC];
    window_max<B, kPairDC>(v2, m2, ia2);
    constexpr int psz = (int)sizeof(PairLinks<AT>);
    const RowView aview = row_view(a.a, a.a_pitch, psz, r2, kPairDC, D);
    const RowView oview = row_view(a.vout, a.v_pitch, 4, r2, kPairDC, D);
    const unsigned int op = (unsigned int)a.v_pitch * 4u;
    // cell j: row r2 + j < D; V_i(x, d) at x = xp - d2 - j in [0, w)
    const int jn = col_ok ? min(kPairDC, D - r2) : 0;
    const int xj = xp - d2;  // x of cell j is xj - j
    const unsigned int ob = (unsigned int)xj * 4u;
    const unsigned int ab2 = (unsigned int)xp * (unsigned int)psz;
    const unsigned int pp = (unsigned int)a.a_pitch * (unsigned int)psz;
#pragma unroll
    for (int j = 0; j < kPairDC; ++j) {
        const bool cell = j < jn;
        const bool live = cell && (unsigned)(xj - j) < (unsigned)w;
        const int val =
            m2[j] >= 0 && (!PIN || a.pin0_x < 0 || xj - j == a.pin0_x) ? hv0[j] + m2[j] : -1;
        const int ra = r2 - B + ia2[j];
        const unsigned int av = (unsigned int)(ra < 0 ? 0 : ra);
        const unsigned int av2 = nxt[wave * kPairDC + ia2[j]][LP + lane];  // the chosen cell's choice
        const unsigned int aoff = cell ? ab2 + j * pp : kOut;
        const unsigned int both = av | (av2 << kLinkBits<AT>);
        if constexpr (sizeof(AT) == 1)
            __builtin_amdgcn_raw_buffer_store_b16((unsigned short)both, aview.rs, (int)aoff, 0, kStoreScope);
        else
            __builtin_amdgcn_raw_buffer_store_b32(both, aview.rs, (int)aoff, 0, kStoreScope);
        __builtin_amdgcn_raw_buffer_store_b32(val, oview.rs, (int)(live ? ob + j * (op - 4u) : kOut),
                                              0, kStoreScope);
    }
}

// Three steps per launch (fixed windows of at most kTriMaxB shifts): the
// two-step scheme one level deeper.  A workgroup owns the cells of step i in
// 64 successor columns x' and 32 displacements, as in dp_pair_fixed.  Those
// read V_{i+1} in the same columns and the displacement rows widened by B;
// these read V_{i+2} at columns x'' = x' + d' and rows widened by 2B, which
// for a displacement row d'' are the 64 + 2B columns x'' - d'' in
// [X0 - B, X0 + 63 + B].  So
//   level 2: V_{i+2} over those cells from V_{i+3} in memory, into LDS stored
//            skewed (column x'' - d'' - X0 + B of row d''), each cell with the
//            row of its window maximum (its choice);
//   level 1: V_{i+1} over the widened rows of the tile from level 2, each cell
//            with its choice and its choice's choice;
//   level 0: step i, writing V_i and at each of its cells the three links of
//            its chain: A_{i+1}, A_{i+2} and A_{i+3} at the same index.
// Level 2 runs in strips of kStrip rows as the pair's phase 1 does: a thread
// owns a column x''' of V_{i+3}, and its cells (x''' - d'', d'') of a strip lie
// on a diagonal; the strip's cells lie in 64 + 2B + 2(kStrip - 1) columns
// x'''.  Level 1 is the pair's phase 1 with the loads of V_{i+2} taken from
// LDS.  About twice the cells of a pair launch for one and a half times its
// steps, and a third of the launches of one step each.  Measured on the
// 4096 x 4096 image (k = 32, bound 8): a wave issues 1465 VALU instructions
// against the pair kernel's 646, and a launch takes 12.3 us against 6.4, so
// ten launches of three steps cost more than fifteen of two; the library
// takes three steps per launch only where a tuning rule asks for them.
constexpr int kTriMaxB = 8;

struct DpTripleJob {
    const int32_t* vin;  // V_{i+3} (or the table H_{k-1}), rows d'''+n-1
    const void* h2;      // H_{i+2} (int32, or uint16 for narrow tables: the kernel's TT)
    const void* h1;      // H_{i+1}
    const void* h0;      // H_i
    int32_t* vout;       // V_i
    void* a2;            // A_{i+3} plane: at each cell of step i, the third link
    void* a1;            // A_{i+2} plane: the second link
    void* a0;            // A_{i+1} plane: the cell's own choice
    int vin_pitch, h_pitch, v_pitch, a_pitch;
    int n, w, items_x, items_y;
    int item0;  // first workgroup of this image in the launch
};

template <int CAP>
struct DpTriplePack {
    DpTripleJob job[CAP];
    int count;
    int stripe;  // column tiles per stripe of the item order
};

template <int B, typename AT, int CAP, typename TT>
__global__ __launch_bounds__(64 * kPairWaves) void dp_triple_fixed(DpTriplePack<CAP> pk) {
    static_assert(B <= kTriMaxB, "three steps per launch take bounds of at most kTriMaxB");
    constexpr int R1 = kPairRows + 2 * B;  // rows of V_{i+1} the workgroup needs
    constexpr int NS1 = (R1 + kStrip - 1) / kStrip;
    constexpr int R2 = kPairRows + 4 * B;  // rows of V_{i+2}
    constexpr int NS2 = (R2 + kStrip - 1) / kStrip;
    constexpr int SC1 = 64 + kStrip - 1;                 // columns x'' of a level-1 strip
    constexpr int SC2 = 64 + 2 * B + 2 * (kStrip - 1);  // columns x''' of a level-2 strip
    constexpr int NV = kStrip + 2 * B;                   // window rows of a strip's cells
    constexpr int NV0 = kPairDC + 2 * B;
    constexpr int esz = (int)sizeof(AT);
    constexpr int LP = kStrip - 1;
    constexpr int LWP = 64 + 2 * LP;  // level-1 row: the tile's columns and padding
    constexpr int P2 = kStrip - 1;
    constexpr int LW2 = 64 + 2 * B + 2 * P2;  // level-2 row (skewed) and padding
    constexpr int ROWS2 = NS1 * kStrip + 2 * B > NS2 * kStrip ? NS1 * kStrip + 2 * B : NS2 * kStrip;
    static_assert(NS1 * SC1 <= 64 * kPairWaves, "level 1 takes one round of the workgroup");
    __shared__ int lv2[ROWS2][LW2];  // V_{i+2}(x'', row g0 + q) at [q][x'' - d'' - X0 + B + P2]
    __shared__ AT ch2[ROWS2][LW2];   // row of that cell's window maximum
    __shared__ int mid[NS1 * kStrip][LWP];  // V_{i+1}(X0 + c, row m0 + q) at [q][LP + c]
    __shared__ AT nx1[NS1 * kStrip][LWP];   // its choice (a row of V_{i+2})
    __shared__ AT nx2[NS1 * kStrip][LWP];   // its choice's choice (a row of V_{i+3})

    // Item order as in dp_pair_fixed: contiguous runs per XCD, walked in
    // stripes of pk.stripe column tiles.
    const int it = xcd_run_item((int)blockIdx.x, (int)gridDim.x);
    int jj = 0;
    if constexpr (CAP > 1) {
        int hi = pk.count - 1;
        while (jj < hi) {
            const int md = (jj + hi + 1) >> 1;
            if (pk.job[md].item0 <= it)
                jj = md;
            else
                hi = md - 1;
        }
    }
    const DpTripleJob& a = pk.job[jj];
    const int n = a.n, w = a.w;
    const int D = 2 * n - 1;
    int bx, by;
    {
        const int local = CAP > 1 ? it - a.item0 : it;
        const int stripe = pk.stripe;
        const int per_stripe = stripe * a.items_y;
        const int st = local / per_stripe, loc = local - st * per_stripe;
        const int sw = min(stripe, a.items_x - st * stripe);
        by = loc / sw;
        bx = st * stripe + (loc - by * sw);
    }
    const int X0 = bx * 64;
    const int r0 = by * kPairRows;  // table row of the first displacement of step i
    const int m0 = r0 - B;          // table row of mid[0]
    const int g0 = r0 - 2 * B;      // table row of lv2[0]
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    constexpr unsigned int hsz = sizeof(TT);
    const unsigned int hp = (unsigned int)a.h_pitch * hsz;

    // Level 0's H_i(x' - d, d) and level 1's H_{i+1}, issued first so that
    // the loads overlap level 2.
    const int xp = X0 + lane;
    const bool col_ok = xp < w;
    const int r2 = r0 + wave * kPairDC;
    const int d2 = r2 - (n - 1);
    const RowView h0v = row_view(a.h0, a.h_pitch, (int)hsz, r2, kPairDC, D);
    const unsigned int h0b = (unsigned int)(r2 - h0v.base) * hp + (unsigned int)(xp - d2) * hsz;
    int hv0[kPairDC];
#pragma unroll
    for (int j = 0; j < kPairDC; ++j) hv0[j] = load_tab<TT>(h0v.rs, h0b + j * (hp - hsz), 0);

    const int t1 = threadIdx.x;  // level-1 task: strip s1, column c1
    const bool has1 = t1 < NS1 * SC1;
    const int s1 = has1 ? t1 / SC1 : 0;
    const int c1 = has1 ? t1 - s1 * SC1 : 0;
    const int q1 = s1 * kStrip;   // mid row of the strip's first displacement
    const int rs1 = m0 + q1;      // its table row
    const int x1s = X0 + rs1 - (n - 1) + c1;  // the strip column x''
    const RowView h1v = row_view(a.h1, a.h_pitch, (int)hsz, m0, R1, D);
    int hv1[kStrip];
    {
        const unsigned int hb =
            (unsigned int)(rs1 - h1v.base) * hp + (unsigned int)(X0 + c1) * hsz;
#pragma unroll
        for (int j = 0; j < kStrip; ++j) hv1[j] = load_tab<TT>(h1v.rs, hb + j * (hp - hsz), 0);
    }

    // Level 2.  Views: V_{i+3} rows [g0 - B, g0 + NS2*kStrip + B), H_{i+2}
    // rows [g0, g0 + NS2*kStrip), each clipped to [0, D).
    const RowView vv = row_view(a.vin, a.vin_pitch, 4, g0 - B, NS2 * kStrip + 2 * B, D);
    const RowView h2v = row_view(a.h2, a.h_pitch, (int)hsz, g0, NS2 * kStrip, D);
    const unsigned int vp = (unsigned int)a.vin_pitch * 4u;
    for (int t = threadIdx.x; t < NS2 * SC2; t += 64 * kPairWaves) {
        const int s = t / SC2, c = t - s * SC2;
        const int q0 = s * kStrip;
        const int rs = g0 + q0;             // table row of the strip's first displacement
        const int ds = rs - (n - 1);        // that displacement
        const int xs = X0 + 2 * ds - B + c;  // the thread's column x''' of V_{i+3}
        const bool xs_ok = (unsigned)xs < (unsigned)w;
        // v[q] = V_{i+3}(x''', row rs - B + q): a cell when the row lies in
        // [0, D) and x''' and x''' plus its displacement lie in [0, w)
        const int rlo = rs - B;
        const int qlo = max(-rlo, (n - 1) - xs - rlo);
        const int qhi = xs_ok ? min(D - rlo, w + (n - 1) - xs - rlo) : qlo;
        // cell j is (x'', row rs + j) with x'' = x''' - ds - j: it exists when
        // the row lies in [0, D), x'' in [0, w) and x''' in [0, w)
        const int jlo = max(-rs, xs - ds - w + 1);
        const int jhi = xs_ok ? min(D - rs, xs - ds + 1) : jlo;
        const unsigned int vb = (unsigned int)(rlo - vv.base) * vp + (unsigned int)xs * 4u;
        const unsigned int hb =
            (unsigned int)(rs - h2v.base) * hp + (unsigned int)(xs - ds) * hsz;
        // cell j lands in column c + P2 - 2j of its row; columns outside the
        // row are cells no later level reads
        const bool inner = qlo <= 0 && qhi >= NV && jlo <= 0 && jhi >= kStrip;
        auto strip = [&](auto inner_tag) {
            constexpr bool INNER = decltype(inner_tag)::value;
            int v[NV];
#pragma unroll
            for (int q = 0; q < NV; ++q) {
                if constexpr (INNER) {
                    v[q] = __builtin_amdgcn_raw_buffer_load_b32(vv.rs, (int)(vb + q * vp), 0, 0);
                } else {
                    const bool ok = q >= qlo && q < qhi;
                    const int tv = __builtin_amdgcn_raw_buffer_load_b32(
                        vv.rs, (int)(ok ? vb + q * vp : kOut), 0, 0);
                    v[q] = ok ? tv : -1;
                }
            }
            int hv[kStrip];
#pragma unroll
            for (int j = 0; j < kStrip; ++j) hv[j] = load_tab<TT>(h2v.rs, hb + j * (hp - hsz), 0);
            __builtin_amdgcn_sched_barrier(0);
            int m[kStrip], ia[kStrip];
            window_max<B, kStrip>(v, m, ia);
#pragma unroll
            for (int j = 0; j < kStrip; ++j) {
                const int col = c + P2 - 2 * j;
                if ((unsigned)col < (unsigned)LW2) {
                    const bool live = INNER || (j >= jlo && j < jhi);
                    lv2[q0 + j][col] = live && m[j] >= 0 ? hv[j] + m[j] : -1;
                    const int ra = rlo + ia[j];  // row of the maximum's d'''
                    ch2[q0 + j][col] = (AT)(INNER || ra >= 0 ? ra : 0);
                }
            }
        };
        if (__builtin_amdgcn_ballot_w64(!inner) == 0)
            strip(std::true_type{});
        else
            strip(std::false_type{});
    }
    __syncthreads();

    // Level 1: the strip column x'' reads V_{i+2}(x'', row rs1 - B + t) at
    // lv2[q1 + t][c1 + 2B - t + P2]; cells (X0 + c1 - j, row rs1 + j).
    if (has1) {
        const int jlo = max(-rs1, X0 + c1 - w + 1);
        const int jhi = (unsigned)x1s < (unsigned)w ? D - rs1 : jlo;
        int v[NV];
        const int* src = &lv2[q1][c1 + 2 * B + P2];
#pragma unroll
        for (int t = 0; t < NV; ++t) v[t] = src[t * (LW2 - 1)];
        int m[kStrip], ia[kStrip];
        window_max<B, kStrip>(v, m, ia);
        int* lrow = &mid[q1][LP + c1];
        AT* nrow1 = &nx1[q1][LP + c1];
        AT* nrow2 = &nx2[q1][LP + c1];
        const AT* csrc = &ch2[q1][c1 + 2 * B + P2];
#pragma unroll
        for (int j = 0; j < kStrip; ++j) {
            const bool live = j >= jlo && j < jhi;
            lrow[j * (LWP - 1)] = live && m[j] >= 0 ? hv1[j] + m[j] : -1;
            const int ra = rs1 - B + ia[j];  // row of the maximum's d''
            nrow1[j * (LWP - 1)] = (AT)(ra >= 0 ? ra : 0);
            nrow2[j * (LWP - 1)] = csrc[ia[j] * (LW2 - 1)];
        }
    }
    __syncthreads();

    // Level 0: step i on the LDS copy of V_{i+1}, as in the pair's phase 2.
    int v0[NV0];
    const int* lcol = &mid[wave * kPairDC][LP + lane];
#pragma unroll
    for (int q = 0; q < NV0; ++q) v0[q] = lcol[q * LWP];
    int m0v[kPairDC], ia0[kPairDC];
    window_max<B, kPairDC>(v0, m0v, ia0);
    const RowView aview = row_view(a.a0, a.a_pitch, esz, r2, kPairDC, D);
    const RowView a1view = row_view(a.a1, a.a_pitch, esz, r2, kPairDC, D);
    const RowView a2view = row_view(a.a2, a.a_pitch, esz, r2, kPairDC, D);
    const RowView oview = row_view(a.vout, a.v_pitch, 4, r2, kPairDC, D);
    const unsigned int op = (unsigned int)a.v_pitch * 4u;
    const unsigned int ap = (unsigned int)a.a_pitch * (unsigned int)esz;
    const int jn = col_ok ? min(kPairDC, D - r2) : 0;
    const int xj = xp - d2;  // x of cell j is xj - j
    const unsigned int ob = (unsigned int)xj * 4u;
    const unsigned int ab = (unsigned int)xp * (unsigned int)esz;
#pragma unroll
    for (int j = 0; j < kPairDC; ++j) {
        const bool cell = j < jn;
        const bool live = cell && (unsigned)(xj - j) < (unsigned)w;
        const int val = m0v[j] >= 0 ? hv0[j] + m0v[j] : -1;
        const int ra = r2 - B + ia0[j];
        const unsigned int av = (unsigned int)(ra < 0 ? 0 : ra);
        const unsigned int av1 = nx1[wave * kPairDC + ia0[j]][LP + lane];
        const unsigned int av2 = nx2[wave * kPairDC + ia0[j]][LP + lane];
        const unsigned int aoff = cell ? ab + j * ap : kOut;
        if constexpr (sizeof(AT) == 1) {
            __builtin_amdgcn_raw_buffer_store_b8((unsigned char)av, aview.rs, (int)aoff, 0, kStoreScope);
            __builtin_amdgcn_raw_buffer_store_b8((unsigned char)av1, a1view.rs, (int)aoff, 0, kStoreScope);
            __builtin_amdgcn_raw_buffer_store_b8((unsigned char)av2, a2view.rs, (int)aoff, 0, kStoreScope);
        } else {
            __builtin_amdgcn_raw_buffer_store_b16((unsigned short)av, aview.rs, (int)aoff, 0, kStoreScope);
            __builtin_amdgcn_raw_buffer_store_b16((unsigned short)av1, a1view.rs, (int)aoff, 0, kStoreScope);
            __builtin_amdgcn_raw_buffer_store_b16((unsigned short)av2, a2view.rs, (int)aoff, 0, kStoreScope);
        }
        __builtin_amdgcn_raw_buffer_store_b32(val, oview.rs, (int)(live ? ob + j * (op - 4u) : kOut),
                                              0, kStoreScope);
    }
}

// Step with per-displacement windows [lo(d), hi(d)] (large mode-0 bounds, the
// angle form, no bound at all).  Both window ends are non-decreasing in d, so
// the windows of a wave's kDCGeneric displacements fall into groups that
// share a point c (c = hi of the group's first window): each window of a
// group is [lo, c] + [c+1, hi].  One descending scan from c gives every
// [lo, c] maximum (recorded as the scan passes each lo) and one ascending scan
// from c+1 gives every [c+1, hi] maximum, so each V cell of the union of the
// windows is read and compared once, with the loads issued eight at a time.
// Ties keep the smallest d' (descending scans take equal values, ascending
// ones only larger values, and the [lo, c] part wins ties).
constexpr int kScanTile = 8;
constexpr int kEmpty = -2147483647 - 1;  // no cell yet (below every V, -1 included)

template <typename AT, int CAP, typename TT>
__global__ __launch_bounds__(64 * kWaves) void dp_step_generic(DpPack<CAP> pk) {
    __shared__ int res_v[kWaves][kDCGeneric][64];
    __shared__ int res_i[kWaves][kDCGeneric][64];
    const int it = xcd_run_item((int)blockIdx.x, (int)gridDim.x);  // as dp_step_fixed
    const int jj = dp_find_job(pk, it);
    const DpJob& a = pk.job[jj];
    const int local = it - a.item0;
    const int bx = local / a.items_y, by = local - bx * a.items_y;
    const int n = a.n, w = a.w;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int xp = bx * 64 + lane;
    const int chunk = by * kWaves + wave;
    const int d0 = -(n - 1) + chunk * kDCGeneric;
    const int D = 2 * n - 1;
    const int jn = min(kDCGeneric, D - (d0 + n - 1));  // displacements of this wave
    const DRange mk = drange(n, xp, vmask(w, a.vin_pin, a.vin_pin_x));
    const bool last = a.key != nullptr;  // no planes to write (views unused)
    const RowView ov = row_view(last ? a.vin : a.vout, a.v_pitch, 4, d0 + n - 1, kDCGeneric, D);
    const RowView av = row_view(last ? a.vin : a.aout, a.a_pitch, sizeof(AT), d0 + n - 1,
                                kDCGeneric, D);
    int hv[kDCGeneric];
#pragma unroll
    for (int j = 0; j < kDCGeneric; ++j) hv[j] = load_h<TT>(a, xp, d0 + j);
    // The wave's windows, one per lane (lanes 0 .. kDCGeneric-1), read back as
    // scalars with readlane: no memory access inside the scans.
    int wlo = 0, whi = 0;
    {
        const int dl = d0 + min(lane, kDCGeneric - 1);
        window_of(n, a.full, a.win, a.bound, min(dl, n - 1), wlo, whi);
    }
    auto lo_of = [&](int j) { return __builtin_amdgcn_readlane(wlo, j); };
    auto hi_of = [&](int j) { return __builtin_amdgcn_readlane(whi, j); };
    if (a.full) {
        // Section 2.2: every window is the whole column, so the workgroup's
        // waves split the column's rows, and the smallest row reaching the
        // maximum wins across them (ties to the lower wave).
        __shared__ int col_v[kWaves][64];
        __shared__ int col_i[kWaves][64];
        const int rows = (D + kWaves - 1) / kWaves;
        const int r_lo = wave * rows, r_hi = min(D, r_lo + rows);
        int cv = kEmpty, ci = 0;
        for (int t0 = r_lo; t0 < r_hi; t0 += kScanTile) {
            int v[kScanTile];
#pragma unroll
            for (int q = 0; q < kScanTile; ++q)
                v[q] = load_v(a.vin, a.vin_pitch, xp, t0 + q - (n - 1), n, mk);
#pragma unroll
            for (int q = 0; q < kScanTile; ++q) {
                const bool take = t0 + q < r_hi && v[q] > cv;
                cv = take ? v[q] : cv;
                ci = take ? t0 + q - (n - 1) : ci;
            }
        }
        col_v[wave][lane] = cv;
        col_i[wave][lane] = ci;
        __syncthreads();
        int m = col_v[0][lane], ia = col_i[0][lane];
#pragma unroll
        for (int q = 1; q < kWaves; ++q) {
            const bool take = col_v[q][lane] > m;
            m = take ? col_v[q][lane] : m;
            ia = take ? col_i[q][lane] : ia;
        }
        Best best;
#pragma unroll
        for (int j = 0; j < kDCGeneric; ++j) {
            if (j >= jn) break;
            emit<AT>(a, ov, av, m, ia + n - 1, hv[j], xp, d0 + j, best);
        }
        finish(a, best, local);
        return;
    }
    for (int ja = 0; ja < jn;) {
        const int c = hi_of(ja);
        int jb = ja;
        while (jb + 1 < jn && lo_of(jb + 1) <= c) ++jb;
        // [lo_j, c], descending; record at each lo_j (j = jb down to ja)
        const int first = lo_of(ja);
        int cv = kEmpty, ci = c;
        int p = jb, plo = lo_of(jb);
        for (int t0 = c; t0 >= first; t0 -= kScanTile) {
            int v[kScanTile];
#pragma unroll
            for (int q = 0; q < kScanTile; ++q) v[q] = load_v(a.vin, a.vin_pitch, xp, t0 - q, n, mk);
#pragma unroll
            for (int q = 0; q < kScanTile; ++q) {
                const int dp = t0 - q;
                if (dp < first) break;
                const bool take = v[q] >= cv;
                cv = take ? v[q] : cv;
                ci = take ? dp : ci;
                while (p >= ja && plo == dp) {
                    res_v[wave][p][lane] = cv;
                    res_i[wave][p][lane] = ci;
                    --p;
                    plo = p >= ja ? lo_of(p) : kEmpty;
                }
            }
        }
        // [c+1, hi_j], ascending; record at each hi_j (j = ja up to jb)
        const int last = hi_of(jb);
        cv = kEmpty;
        ci = c;
        p = ja;
        int phi = hi_of(ja);
        auto record_up = [&](int at) {
            while (p <= jb && phi == at) {
                const int sv = res_v[wave][p][lane];
                const bool up = cv > sv;  // the [lo, c] part wins ties
                res_v[wave][p][lane] = up ? cv : sv;
                if (up) res_i[wave][p][lane] = ci;
                ++p;
                phi = p <= jb ? hi_of(p) : kEmpty;
            }
        };
        record_up(c);
        for (int t0 = c + 1; t0 <= last; t0 += kScanTile) {
            int v[kScanTile];
#pragma unroll
            for (int q = 0; q < kScanTile; ++q) v[q] = load_v(a.vin, a.vin_pitch, xp, t0 + q, n, mk);
#pragma unroll
            for (int q = 0; q < kScanTile; ++q) {
                const int dp = t0 + q;
                if (dp > last) break;
                const bool take = v[q] > cv;
                cv = take ? v[q] : cv;
                ci = take ? dp : ci;
                record_up(dp);
            }
        }
        ja = jb + 1;
    }
    Best best;
#pragma unroll
    for (int j = 0; j < kDCGeneric; ++j) {
        if (j >= jn) break;
        const int m = res_v[wave][j][lane];
        const int ia = res_i[wave][j][lane];
        emit<AT>(a, ov, av, m, ia + n - 1, hv[j], xp, d0 + j, best);
    }
    finish(a, best, local);
}

// Step with per-displacement windows for bands of at most 255 displacements
// and no pin (the angle form, mode-0 bounds above 16): a workgroup owns
// kBlkCols successor columns x' and every displacement row, so each cell of
// V_{i+1} is loaded once, into LDS, however many windows hold it.  The rows
// are cut into blocks of kBlk; per column the workgroup keeps the maxima
// from each block's start down to every row (prefix) and from every row to
// its block's end (suffix), each with the smallest row reaching it, and a
// sparse table of the block maxima over 1, 2, 4 and 8 consecutive blocks.
// A window [lo, hi] inside one block is scanned directly (at most kBlk
// cells); one that crosses blocks is the suffix at lo, at most two
// overlapping runs of whole blocks, and the prefix at hi, taken in that
// order with a later candidate winning only when larger, so ties keep the
// smallest d' as everywhere else.
constexpr int kBlkCols = 16;      // successor columns per workgroup
constexpr int kBlk = 16;          // rows per block
constexpr int kBlkRows = 256;     // rows held: D <= 255
constexpr int kBlkLevels = 4;     // block runs of 1, 2, 4 and 8
constexpr int kBlkThreads = 1024; // 16 waves: four per SIMD hide the LDS round trips
constexpr int kBlkLanes = kBlkThreads / kBlkCols;  // row lanes
constexpr int kBlkOut = kBlkRows / kBlkLanes;      // rows (cells) per thread

template <typename AT, int CAP, typename TT>
__global__ __launch_bounds__(kBlkThreads) void dp_step_blocks(DpPack<CAP> pk) {
    constexpr int NB = kBlkRows / kBlk;
    static_assert(NB * kBlkCols <= kBlkThreads, "one block scan per thread");
    __shared__ int vt[kBlkRows][kBlkCols];       // V_{i+1}(X0 + c, row r), -1 where none
    __shared__ int pre_v[kBlkRows][kBlkCols];    // max over [block start, r]
    __shared__ int suf_v[kBlkRows][kBlkCols];    // max over [r, block end]
    __shared__ unsigned char pre_i[kBlkRows][kBlkCols];  // its smallest row
    __shared__ unsigned char suf_i[kBlkRows][kBlkCols];
    __shared__ int run_v[kBlkLevels][NB][kBlkCols];  // max over blocks [b, b + 2^l)
    __shared__ unsigned char run_i[kBlkLevels][NB][kBlkCols];
    __shared__ unsigned char wlo[kBlkRows], whi[kBlkRows];  // window of each row, as rows

    const int it = xcd_run_item((int)blockIdx.x, (int)gridDim.x);
    const int jj = dp_find_job(pk, it);
    const DpJob& a = pk.job[jj];
    const int local = it - a.item0;  // the column tile
    const int n = a.n, w = a.w, D = 2 * n - 1;
    const int t = threadIdx.x;
    const int c = t & (kBlkCols - 1);
    const int rq = t / kBlkCols;  // first row of the thread's rows rq, rq + kBlkLanes, ...
    const int xp = local * kBlkCols + c;

    if (t < D) {
        int lo, hi;
        window_of(n, a.full, a.win, a.bound, t - (n - 1), lo, hi);
        wlo[t] = (unsigned char)(lo + n - 1);
        whi[t] = (unsigned char)(hi + n - 1);
    }
    // H_i(x' - d, d) of the thread's cells, then its rows of V_{i+1}
    int hv[kBlkOut];
#pragma unroll
    for (int j = 0; j < kBlkOut; ++j) hv[j] = load_h<TT>(a, xp, rq + kBlkLanes * j - (n - 1));
    const DRange mk = drange(n, xp, VMask{0, w, 0, w});
#pragma unroll
    for (int j = 0; j < kBlkOut; ++j) {
        const int r = rq + kBlkLanes * j;
        vt[r][c] = load_v(a.vin, a.vin_pitch, xp, r - (n - 1), n, mk);  // -1 past row D-1
    }
    __syncthreads();
    if (rq < NB) {
        // block rq of column c: prefix maxima ascending (ties keep the first),
        // suffix maxima descending (ties move to the smaller row)
        const int r0 = rq * kBlk;
        int pv = kEmpty, pi = r0;
#pragma unroll
        for (int q = 0; q < kBlk; ++q) {
            const int v = vt[r0 + q][c];
            const bool take = v > pv;
            pv = take ? v : pv;
            pi = take ? r0 + q : pi;
            pre_v[r0 + q][c] = pv;
            pre_i[r0 + q][c] = (unsigned char)pi;
        }
        int sv = kEmpty, si = r0 + kBlk - 1;
#pragma unroll
        for (int q = kBlk - 1; q >= 0; --q) {
            const int v = vt[r0 + q][c];
            const bool take = v >= sv;
            sv = take ? v : sv;
            si = take ? r0 + q : si;
            suf_v[r0 + q][c] = sv;
            suf_i[r0 + q][c] = (unsigned char)si;
        }
        run_v[0][rq][c] = sv;
        run_i[0][rq][c] = (unsigned char)si;
    }
    __syncthreads();
    if (rq < NB) {
        // runs of 2, 4, 8 blocks from block rq, ascending (ties keep the first)
        int mv = run_v[0][rq][c], mi = run_i[0][rq][c];
#pragma unroll
        for (int l = 1; l < kBlkLevels; ++l) {
#pragma unroll
            for (int b = (1 << (l - 1)); b < (1 << l); ++b) {
                const int bb = min(rq + b, NB - 1);
                const int v = run_v[0][bb][c];
                const bool take = rq + b < NB && v > mv;
                mv = take ? v : mv;
                mi = take ? run_i[0][bb][c] : mi;
            }
            run_v[l][rq][c] = mv;
            run_i[l][rq][c] = (unsigned char)mi;
        }
    }
    __syncthreads();

    const bool last = a.key != nullptr;  // the image's last step: keys, no planes
    const RowView ov = row_view(last ? a.vin : a.vout, a.v_pitch, 4, 0, D, D);
    const RowView av = row_view(last ? a.vin : a.aout, a.a_pitch, sizeof(AT), 0, D, D);
    const bool col = xp < w;
    Best best;
#pragma unroll
    for (int j = 0; j < kBlkOut; ++j) {
        const int r = rq + kBlkLanes * j;
        if (r >= D) break;
        const int lo = wlo[r], hi = whi[r];
        const int bl = lo / kBlk, bh = hi / kBlk;
        int m, ia;
        if (bl == bh) {
            m = kEmpty;
            ia = lo;
            for (int q = lo; q <= hi; ++q) {
                const int v = vt[q][c];
                const bool take = v > m;
                m = take ? v : m;
                ia = take ? q : ia;
            }
        } else {
            m = suf_v[lo][c];
            ia = suf_i[lo][c];
            const int cnt = bh - bl - 1;  // whole blocks between
            if (cnt > 0) {
                const int l = 31 - __builtin_clz((unsigned)cnt);
                const int v1 = run_v[l][bl + 1][c], v2 = run_v[l][bh - (1 << l)][c];
                const bool t1 = v1 > m;
                m = t1 ? v1 : m;
                ia = t1 ? run_i[l][bl + 1][c] : ia;
                const bool t2 = v2 > m;
                m = t2 ? v2 : m;
                ia = t2 ? run_i[l][bh - (1 << l)][c] : ia;
            }
            const int vp = pre_v[hi][c];
            const bool tp = vp > m;
            m = tp ? vp : m;
            ia = tp ? pre_i[hi][c] : ia;
        }
        if (!col) continue;
        if (last) {
            const int x = xp - (r - (n - 1));
            if ((unsigned)x < (unsigned)w) take_best(best, pack_key(m >= 0 ? hv[j] + m : -1, x, r, D), ia);
            continue;
        }
        const unsigned int aoff = (unsigned int)r * a.a_pitch * sizeof(AT) + (unsigned int)xp * sizeof(AT);
        if constexpr (sizeof(AT) == 1)
            __builtin_amdgcn_raw_buffer_store_b8((unsigned char)ia, av.rs, (int)aoff, 0, kStoreScope);
        else
            __builtin_amdgcn_raw_buffer_store_b16((unsigned short)ia, av.rs, (int)aoff, 0, kStoreScope);
        const int x = xp - (r - (n - 1));
        if ((unsigned)x < (unsigned)w) {
            const int val = m >= 0 ? hv[j] + m : -1;
            __builtin_amdgcn_raw_buffer_store_b32(
                val, ov.rs, (int)((unsigned int)r * a.v_pitch * 4u + (unsigned int)x * 4u), 0,
                kStoreScope);
        }
    }
    if (last) {
        // the workgroup's best key and that cell's successor, slot = column tile
        constexpr int W = kBlkThreads / 64;
        __shared__ unsigned long long part[W];
        __shared__ int part_s[W];
        const int lane = t & 63, wave = t >> 6;
        best = wave_best(best);
        if (lane == 0) {
            part[wave] = best.key;
            part_s[wave] = best.succ;
        }
        __syncthreads();
        if (t == 0) {
            unsigned long long mk2 = part[0];
            int ms = part_s[0];
#pragma unroll
            for (int q = 1; q < W; ++q) {
                const bool tk = part[q] > mk2;
                mk2 = tk ? part[q] : mk2;
                ms = tk ? part_s[q] : ms;
            }
            a.key[local] = mk2;
            a.succ[local] = ms;
        }
    }
}

// k = 1: the answer is the best masked cell of H_0 (htab), pinned as vin.
template <int CAP>
__global__ __launch_bounds__(64 * kWaves) void argmax_table(DpPack<CAP> pk) {
    const int jj = dp_find_job(pk, blockIdx.x);
    const DpJob& a = pk.job[jj];
    const int local = blockIdx.x - a.item0;
    const int bx = local % a.items_x, by = local / a.items_x;
    const int n = a.n, w = a.w;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int x = bx * 64 + lane;
    const int chunk = by * kWaves + wave;
    const int D = 2 * n - 1;
    const VMask mk = vmask(w, a.vin_pin, a.vin_pin_x);
    Best best;  // k = 1: no successor
    for (int j = 0; j < kDCGeneric; ++j) {
        const int r = chunk * kDCGeneric + j;
        const int d = r - (n - 1);
        if (r >= D || (unsigned)(x - mk.xlo) >= (unsigned)mk.xlen ||
            (unsigned)(x + d - mk.tlo) >= (unsigned)mk.tlen)
            continue;
        take_best(best, pack_key(static_cast<const int32_t*>(a.htab)[(size_t)r * a.h_pitch + x], x, r, D), 0);
    }
    finish(a, best, local);
}

// Three bands of the walk in one memory round trip, for windows of at most
// 31 displacements: with x_i and d_i known, read A_{i+1}(x_{i+1}, d_i), every
// candidate A_{i+2}(x_{i+1} + d', d') for d' in the window of d_i (one per
// lane), and every candidate A_{i+3} for d'' in the window of each d' (lanes
// 0-31 take the even d' of the window, lanes 32-63 the odd ones, U loads per
// lane).  Candidate indices are clamped into the planes rather than masked:
// the candidate that is finally selected is always inside, and what the
// others read is never used.  Returns false when a link leaves the image (the
// caller reports no polyline).
template <typename AT, int U>
__device__ __forceinline__ bool walk_three(const WalkJob& a, int lane, int& x, int& r, int& i) {
    const int n = a.n, w = a.w, D = 2 * n - 1;
    const int B = a.bound, L1 = 2 * B + 1;
    const unsigned int pitch = (unsigned int)a.a_pitch;
    const int xn = x + r - (n - 1);
    if (xn < 0 || xn >= w || r < 0 || r >= D) return false;
    const AT* P1 = static_cast<const AT*>(a.a_base) + (size_t)(i - 1) * a.a_plane;  // A_{i+1}
    const AT* P2 = P1 + a.a_plane;                                                  // A_{i+2}
    const AT* P3 = P2 + a.a_plane;                                                  // A_{i+3}
    const int rn_v = P1[(unsigned int)r * pitch + (unsigned int)xn];
    int s1;
    {
        const int c1 = min(max(r - B + lane, 0), D - 1);
        const int x2 = min(max(xn + c1 - (n - 1), 0), w - 1);
        s1 = P2[(unsigned int)c1 * pitch + (unsigned int)x2];
    }
    const int l2 = lane & 31;
    int s2[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int c1 = r - B + 2 * u + (lane >> 5);
        const int c2 = min(max(c1 - B + l2, 0), D - 1);
        const int x3 = min(max(xn + c1 + c2 - 2 * (n - 1), 0), w - 1);
        s2[u] = P3[(unsigned int)c2 * pitch + (unsigned int)x3];
    }
    // No branch until every load of the round trip has been issued and used:
    // an early exit here would let the compiler sink the candidate loads
    // behind the first one, two memory latencies per trip instead of one.
    // Every lane loaded the same pointer: as a wave-uniform value it lets the
    // candidates be picked by v_readlane with a scalar lane index rather than
    // by a permute through the LDS unit.
    const int rn = __builtin_amdgcn_readfirstlane(rn_v);
    const int l1 = rn - (r - B);
    const bool ok1 = (unsigned)l1 < (unsigned)L1 && rn < D;
    const int xnn = xn + rn - (n - 1);
    const int r2 = __builtin_amdgcn_readlane(s1, l1 & 63);
    const int l2s = r2 - (rn - B);
    const bool ok2 = ok1 && xnn >= 0 && xnn < w && (unsigned)l2s < (unsigned)L1 && r2 >= 0 && r2 < D;
    const int x3 = xnn + r2 - (n - 1);
    const bool ok3 = ok2 && x3 >= 0 && x3 < w;
    const int slot = l1 >> 1;
    int mine = s2[0];
#pragma unroll
    for (int u = 1; u < U; ++u) mine = slot == u ? s2[u] : mine;
    const int r3 = __builtin_amdgcn_readlane(mine, ((l1 & 1) << 5) | (l2s & 31));
    if (lane == 0) {
        if (ok1) a.xs[i + 1] = xn;
        if (ok2) a.xs[i + 2] = xnn;
        if (ok3) a.xs[i + 3] = x3;
    }
    if (!ok3) return false;
    x = x3;
    r = r3;
    i += 3;
    return true;
}

// Four bands per round trip over the pairs of steps made in one launch each
// (from i = 1 while i + 3 <= pair_top), windows of at most 31 displacements.
// A pair's plane gives both of its links at the index of its lower band's
// cell, so with x_i and d_i known one load gives d_{i+1} and d_{i+2}; in the
// same round trip the next pair's links are loaded for every candidate
// (d_{i+1}, d_{i+2}) = (d_i - B + q1, d_i - 2B + q1 + q2), q1, q2 in [0, L1):
// candidate t = q1 * L1 + q2 is slot t / 64 of lane t % 64, so U slots cover
// the L1 * L1 candidates.  Loads are buffer loads through views of the rows a
// round trip can reach (row d_i of one pair, rows d_i - 2B .. d_i + 2B of the
// next): a candidate whose index leaves its view reads 0 instead of faulting,
// and the one finally selected always lies inside.  Returns false when a link
// leaves the image (the caller reports no polyline).
template <typename AT, int U>
__device__ __forceinline__ bool walk_fours(const WalkJob& a, int lane, int& x, int& r, int& i) {
    using PT = PairLinks<AT>;
    constexpr unsigned int lo_mask = (1u << kLinkBits<AT>) - 1u;
    constexpr unsigned int psz = sizeof(PT);
    const int n = a.n, w = a.w, D = 2 * n - 1;
    const int B = a.bound, L1 = 2 * B + 1;
    const unsigned int pitch = (unsigned int)a.a_pitch;
    // this lane's candidates: q1 (the window position of d_{i+1}) and the row
    // offset q1 + q2 - 2B of d_{i+2} from d_i, fixed for the whole walk
    int q1[U], dq[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int t = u * 64 + lane;
        q1[u] = t / L1;
        dq[u] = t - q1[u] * (L1 - 1) - 2 * B;  // q1 + q2 - 2B with q2 = t - q1 * L1
    }
    const AT* A = static_cast<const AT*>(a.a_base);
    while (i + 3 <= a.pair_top) {
        const int xn = x + r - (n - 1);
        if (xn < 0 || xn >= w || r < 0 || r >= D) return false;
        const RowView v12 = row_view(A + (size_t)(i - 1) * a.a_plane, a.a_pitch, psz, r, 1, D);
        const RowView v34 = row_view(A + (size_t)(i + 1) * a.a_plane, a.a_pitch, psz, r - 2 * B,
                                     4 * B + 1, D);
        const unsigned int off = (unsigned int)xn * psz;
        unsigned int p12;
        if constexpr (psz == 2)
            p12 = __builtin_amdgcn_raw_buffer_load_b16(v12.rs, (int)off, 0, 0);
        else
            p12 = __builtin_amdgcn_raw_buffer_load_b32(v12.rs, (int)off, 0, 0);
        // candidate cell of the next pair: row c2 = r + dq, column
        // x_{i+3} = xn + d_{i+1} + d_{i+2} with d_{i+1} = r - B + q1 - (n - 1)
        // (offsets relative to the view's first row; a row before it wraps to
        // a huge offset, one past its end lies beyond its records)
        const int base_x = xn + 2 * r - B - 2 * (n - 1);
        const int rel = r - v34.base;
        unsigned int s34[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int c2 = rel + dq[u];
            const int x3 = base_x + q1[u] + dq[u];
            const unsigned int o3 = ((unsigned int)c2 * pitch + (unsigned int)x3) * psz;
            if constexpr (psz == 2)
                s34[u] = __builtin_amdgcn_raw_buffer_load_b16(v34.rs, (int)o3, 0, 0);
            else
                s34[u] = __builtin_amdgcn_raw_buffer_load_b32(v34.rs, (int)o3, 0, 0);
        }
        // No branch until the loads have been used; the pair every lane
        // loaded alike is taken as a wave-uniform value.
        const unsigned int p12u = __builtin_amdgcn_readfirstlane(p12);
        const int rn = (int)(p12u & lo_mask);
        const int r2 = (int)(p12u >> kLinkBits<AT>);
        const int l1 = rn - (r - B);
        const bool ok1 = (unsigned)l1 < (unsigned)L1 && rn < D;
        const int xnn = xn + rn - (n - 1);
        const int l2s = r2 - (rn - B);
        const bool ok2 = ok1 && xnn >= 0 && xnn < w && (unsigned)l2s < (unsigned)L1 && r2 >= 0 && r2 < D;
        const int x3 = xnn + r2 - (n - 1);
        const bool ok3 = ok2 && x3 >= 0 && x3 < w;
        const int tsel = l1 * L1 + l2s;  // the candidate that was taken
        const int slot = tsel >> 6;
        unsigned int m34 = s34[0];
#pragma unroll
        for (int u = 1; u < U; ++u) m34 = slot == u ? s34[u] : m34;
        const unsigned int p34 = __builtin_amdgcn_readlane(m34, tsel & 63);
        const int r3 = (int)(p34 & lo_mask);
        const int r4 = (int)(p34 >> kLinkBits<AT>);
        const int l3 = r3 - (r2 - B);
        const int x4 = x3 + r3 - (n - 1);
        const bool ok4 = ok3 && (unsigned)l3 < (unsigned)L1 && r3 >= 0 && r3 < D && x4 >= 0 && x4 < w;
        if (lane == 0) {
            if (ok1) a.xs[i + 1] = xn;
            if (ok2) a.xs[i + 2] = xnn;
            if (ok3) a.xs[i + 3] = x3;
            if (ok4) a.xs[i + 4] = x4;
        }
        if (!ok4) return false;
        x = x4;
        r = r4;
        i += 4;
    }
    return true;
}

// Walk of eq. (5), one wave per image: reduce the workgroup keys of the last
// step, then follow the back-pointers.  The walk is a chain of dependent
// loads, so every load is unconditional (clamped index, result masked) and
// the loads of one round trip are all issued before the first is used.
template <typename AT, int CAP>
__global__ __launch_bounds__(64) void walk(WalkPack<CAP> pk) {
    const WalkJob& a = pk.job[blockIdx.x];
    const int lane = threadIdx.x;
    const int n = a.n, w = a.w, k = a.k;
    const int D = 2 * n - 1;
    // The keys of the last step and, with each, the successor of that cell.
    Best bk;
    for (int q0 = 0; q0 < a.n_keys; q0 += 64 * 8) {
        unsigned long long t[8];
        int sc[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int q = q0 + u * 64 + lane;
            t[u] = a.key[q < a.n_keys ? q : 0];
            sc[u] = a.succ[q < a.n_keys ? q : 0];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const bool tk = t[u] > bk.key;
            bk.key = tk ? t[u] : bk.key;
            bk.succ = tk ? sc[u] : bk.succ;
        }
    }
    bk = wave_best(bk);
    const unsigned long long kv = bk.key;
    const unsigned int lin = 0xffffffffu - (unsigned int)(kv & 0xffffffffull);
    const unsigned int xu = lin / (unsigned int)D;
    int x = (int)xu;
    int r = (int)(lin % (unsigned int)D);
    if ((kv >> 32) == 0 || xu >= (unsigned int)w) {
        if (lane == 0) *a.score = -1;
        return;
    }
    if (lane == 0) a.xs[0] = x;
    if (k >= 2) {
        // First successor: recorded by the last step with the cell's key (the
        // smallest d' of its window reaching the maximum of V_1).
        const int x1 = x + r - (n - 1);
        if (x1 < 0 || x1 >= w) {
            if (lane == 0) *a.score = -1;
            return;
        }
        const int r1 = bk.succ;
        if (lane == 0) a.xs[1] = x1;
        x = x1;
        r = r1;
        // Later successors from the stored planes: three bands per round trip
        // for windows of at most 31 displacements (walk_three), else two: with
        // link i known,
        // read A_{i+1}(x_{i+1}, d_i) and, for every possible d_{i+1}
        // (lane-strided), A_{i+2}(x_{i+1} + d_{i+1}, d_{i+1}).
        const AT* A = static_cast<const AT*>(a.a_base);
        const unsigned int pitch = (unsigned int)a.a_pitch;
        const int L1 = 2 * a.bound + 1;
        const bool narrow = !a.full && a.win == nullptr && L1 <= 31;
        int i = 1;
        while (i + 1 < k) {
            if (i + 2 <= a.tri_top) {
                // three links made in one launch (see WalkJob::tri_top)
                const int xn = x + r - (n - 1);
                if (xn < 0 || xn >= w || r < 0 || r >= D) {
                    if (lane == 0) *a.score = -1;
                    return;
                }
                const AT* Pi = A + (size_t)(i - 1) * a.a_plane;
                const unsigned int off = (unsigned int)r * pitch + (unsigned int)xn;
                const int rn = __builtin_amdgcn_readfirstlane((int)Pi[off]);
                const int r2 = __builtin_amdgcn_readfirstlane((int)Pi[a.a_plane + off]);
                const int r3 = __builtin_amdgcn_readfirstlane((int)Pi[2 * a.a_plane + off]);
                const int xnn = xn + rn - (n - 1);
                const int x3 = xnn + r2 - (n - 1);
                if (rn >= D || r2 >= D || xnn < 0 || xnn >= w || x3 < 0 || x3 >= w) {
                    if (lane == 0) *a.score = -1;
                    return;
                }
                if (lane == 0) {
                    a.xs[i + 1] = xn;
                    a.xs[i + 2] = xnn;
                    a.xs[i + 3] = x3;
                }
                x = x3;
                r = r3;
                i += 3;
                continue;
            }
            if (i >= a.pair_lo && !((i - a.pair_lo) & 1) && i < a.pair_top) {
                // a pair of links made in one launch (see WalkJob::pair_top)
                if (narrow && a.pair_lo == 1 && i + 3 <= a.pair_top) {
                    // U slots of 64 candidates cover L1 * L1.  Past 16 slots
                    // (L1 = 33) the gathers of one round trip cost more than
                    // the round trips saved, and two bands per trip are faster.
                    const bool ok = L1 <= 7    ? walk_fours<AT, 1>(a, lane, x, r, i)
                                    : L1 <= 11 ? walk_fours<AT, 2>(a, lane, x, r, i)
                                    : L1 <= 17 ? walk_fours<AT, 5>(a, lane, x, r, i)
                                    : L1 <= 23 ? walk_fours<AT, 9>(a, lane, x, r, i)
                                               : walk_fours<AT, 16>(a, lane, x, r, i);
                    if (!ok) {
                        if (lane == 0) *a.score = -1;
                        return;
                    }
                    continue;
                }
                const int xn = x + r - (n - 1);
                if (xn < 0 || xn >= w || r < 0 || r >= D) {
                    if (lane == 0) *a.score = -1;
                    return;
                }
                const PairLinks<AT>* Pi =
                    reinterpret_cast<const PairLinks<AT>*>(A + (size_t)(i - 1) * a.a_plane);
                const unsigned int both = __builtin_amdgcn_readfirstlane(
                    (unsigned int)Pi[(unsigned int)r * pitch + (unsigned int)xn]);
                const int rn = (int)(both & ((1u << kLinkBits<AT>) - 1u));
                const int r2 = (int)(both >> kLinkBits<AT>);
                const int xnn = xn + rn - (n - 1);
                if (rn >= D || xnn < 0 || xnn >= w) {
                    if (lane == 0) *a.score = -1;
                    return;
                }
                if (lane == 0) {
                    a.xs[i + 1] = xn;
                    a.xs[i + 2] = xnn;
                }
                x = xnn;
                r = r2;
                i += 2;
                continue;
            }
            if (narrow && i + 3 < k) {
                const bool ok = L1 <= 7    ? walk_three<AT, 4>(a, lane, x, r, i)
                                : L1 <= 11 ? walk_three<AT, 6>(a, lane, x, r, i)
                                : L1 <= 17 ? walk_three<AT, 9>(a, lane, x, r, i)
                                : L1 <= 23 ? walk_three<AT, 12>(a, lane, x, r, i)
                                           : walk_three<AT, 16>(a, lane, x, r, i);
                if (!ok) {
                    if (lane == 0) *a.score = -1;
                    return;
                }
                continue;
            }
            const int xn = x + r - (n - 1);
            if (xn < 0 || xn >= w || r < 0 || r >= D) {
                if (lane == 0) *a.score = -1;
                return;
            }
            const AT* Pi = A + (size_t)(i - 1) * a.a_plane;
            const int rn_v = Pi[(unsigned int)r * pitch + (unsigned int)xn];
            const bool two = (i + 2 < k) && D <= 256;
            int spec[4];
            if (two) {
                const AT* Pn = A + (size_t)i * a.a_plane;
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int c = lane + 64 * j;
                    const int xc = xn + c - (n - 1);
                    const bool ok = c < D && xc >= 0 && xc < w;
                    const int v = Pn[ok ? (unsigned int)c * pitch + (unsigned int)xc : 0u];
                    spec[j] = ok ? v : 0;
                }
            }
            const int rn = __builtin_amdgcn_readfirstlane(rn_v);  // the same in every lane
            if (rn >= D) {
                if (lane == 0) *a.score = -1;
                return;
            }
            if (lane == 0) a.xs[i + 1] = xn;
            if (two) {
                const int xnn = xn + rn - (n - 1);
                if (xnn < 0 || xnn >= w) {
                    if (lane == 0) *a.score = -1;
                    return;
                }
                const int slot = rn >> 6;
                const int mine = slot == 0 ? spec[0] : slot == 1 ? spec[1] : slot == 2 ? spec[2] : spec[3];
                const int r2 = __builtin_amdgcn_readlane(mine, rn & 63);
                if (lane == 0) a.xs[i + 2] = xnn;
                x = xnn;
                r = r2;
                i += 2;
            } else {
                x = xn;
                r = rn;
                i += 1;
            }
        }
        if (r < 0 || r >= D) {
            if (lane == 0) *a.score = -1;
            return;
        }
    }
    if (lane == 0) {
        a.xs[k] = x + r - (n - 1);
        *a.score = (int)(kv >> 32) - 1;
    }
}

// Mode-1 windows: lo(d) and hi(d) bracket every d' with n*|d'-d| <= t*(n*n + d*d').
// One wave per d: the lanes test 64 candidates d' at a time and the first
// and last admissible ones come from the wave's ballot.  Both sides of the
// test are exact products of integers below 2^22 except the one rounding of
// t times the integer, so the result does not depend on how the compiler
// groups the arithmetic.
__global__ __launch_bounds__(64) void angle_windows(int n, double t, int32_t* __restrict__ win) {
    const int D = 2 * n - 1;
    const int r = blockIdx.x;
    const int lane = threadIdx.x;
    const int d = r - (n - 1);
    int lo = n, hi = -n;
    for (int q0 = 0; q0 < D; q0 += 64) {
        const int q = q0 + lane;
        const int dp = q - (n - 1);
        const double lhs = (double)n * (double)abs(dp - d);
        const double rhs = t * ((double)n * (double)n + (double)d * (double)dp);
        const unsigned long long m = __builtin_amdgcn_ballot_w64(q < D && lhs <= rhs);
        if (m) {
            if (lo == n) lo = q0 + (int)__builtin_ctzll(m) - (n - 1);
            hi = q0 + 63 - (int)__builtin_clzll(m) - (n - 1);
        }
    }
    if (lane == 0) {
        win[r] = lo;
        win[D + r] = hi;
    }
}

// ---- unbounded bend: the column-maximum recurrence ---------------------------
//
// With every bend admissible (no restriction of Section 2.3), the range
// maximum of eq. (3) runs over every d', so the best continuation
// M_{i+1}(x', d) = max_{d'} V_{i+1}(x', d') does not depend on d.  Writing
// U_i(x) for that column maximum of V_i,
//
//   U_i(x) = max over d with x + d in [0, w) of H_i(x, d) + U_{i+1}(x + d),
//
// with U_k = 0 (V_{k-1} is the table wherever x + d stays in the image), and
// the back-pointer A_{i+1}(x', d) is the same for every d: the smallest d'
// reaching U_{i+1}(x').  So a step keeps one value and one back-pointer per
// column, B_i(x) = that smallest d (as its row d + n - 1), instead of the
// planes of V_i and A_{i+1}: it reads the table once and U_{i+1} (w values,
// from cache) and writes 5 bytes per column.  The last step (band 0) reduces
// U_0 to one packed key per workgroup (largest value, then smallest x); the
// walk takes x_0 from the keys and follows x_{i+1} = x_i + d_i with
// d_i = B_i(x_i).  The greedy smallest index at every step gives the
// lexicographically smallest optimal polyline, as in the other kernels.
//
// Layout: a workgroup owns 64 columns x (one per lane, coalesced loads) and
// its kColWaves waves split the displacement rows, each scanning its rows in
// ascending order; the waves' partial maxima meet in LDS, lowest rows first.
constexpr int kColWaves = 16;

struct ColJob {
    const void* htab;         // H_i (the kernel's TT; int32 for band k-1)
    const int32_t* uin;       // U_{i+1}, or null on band k-1 (U_k = 0)
    int32_t* uout;            // U_i, or null on band 0
    void* bout;               // B_i: the row of each column's smallest maximizing d
    unsigned long long* key;  // band 0: one packed key per workgroup, else null
    int h_pitch;
    int n, w;
    int item0;  // first workgroup of this image in the launch
};

template <int CAP>
struct ColPack {
    ColJob job[CAP];
    int count;
};

__device__ __forceinline__ unsigned long long col_key(int val, int x) {
    return ((unsigned long long)(unsigned int)(val + 1) << 32) |
           (unsigned long long)(0xffffffffu - (unsigned int)x);
}

template <typename AT, int CAP, typename TT>
__global__ __launch_bounds__(64 * kColWaves) void dp_colmax(ColPack<CAP> pk) {
    const int it = xcd_run_item((int)blockIdx.x, (int)gridDim.x);
    int jj = 0;
    if constexpr (CAP > 1) {
        int hi = pk.count - 1;
        while (jj < hi) {
            const int md = (jj + hi + 1) >> 1;
            if (pk.job[md].item0 <= it)
                jj = md;
            else
                hi = md - 1;
        }
    }
    const ColJob& a = pk.job[jj];
    const int n = a.n, w = a.w, D = 2 * n - 1;
    const int tile = CAP > 1 ? it - a.item0 : it;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int x = tile * 64 + lane;
    const bool col = x < w;
    const int R = (D + kColWaves - 1) / kColWaves;
    const int r0 = wave * R, r1 = min(r0 + R, D);
    const TT* H = static_cast<const TT*>(a.htab);
    int best = kEmpty, brow = 0;
    for (int rb = r0; rb < r1; rb += 8) {
        int hv[8], uv[8];
        bool ok[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int r = rb + j;
            const int xt = x + r - (n - 1);  // successor column x + d
            ok[j] = col && r < r1 && (unsigned)xt < (unsigned)w;
            const size_t off = ok[j] ? (size_t)r * (size_t)a.h_pitch + (size_t)x : 0;
            hv[j] = (int)H[off];
            uv[j] = a.uin ? a.uin[ok[j] ? xt : 0] : 0;
        }
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int v = hv[j] + uv[j];
            const bool t = ok[j] && v > best;  // ascending rows: ties keep the smaller d
            best = t ? v : best;
            brow = t ? rb + j : brow;
        }
    }
    __shared__ int pv[kColWaves][64];
    __shared__ int pr[kColWaves][64];
    pv[wave][lane] = best;
    pr[wave][lane] = brow;
    __syncthreads();
    if (wave != 0) return;
    // waves hold ascending row ranges: a later wave wins only when larger
    int b = pv[0][lane], r = pr[0][lane];
#pragma unroll
    for (int q = 1; q < kColWaves; ++q) {
        const bool t = pv[q][lane] > b;
        b = t ? pv[q][lane] : b;
        r = t ? pr[q][lane] : r;
    }
    if (col) {
        static_cast<AT*>(a.bout)[x] = (AT)r;
        if (a.uout) a.uout[x] = b;
    }
    if (a.key) {
        const unsigned long long kk = wave_max_u64(col ? col_key(b, x) : 0ull);
        if (lane == 0) a.key[tile] = kk;
    }
}

// Walk of the column recurrence, one wave per image: x_0 from the keys, then
// d_i = B_i(x_i), several bands per memory round trip: with x_i known, a trip
// loads B_i(x_i), B_{i+1} at every column x_i + d the first link can reach
// (U1 per lane) and, when U2 > 0, B_{i+2} at every column x_i + s the first
// two can reach (U2 per lane), and resolves three bands (two when U2 = 0)
// with lane reads.  Loads are clamped into the rows and the image; what an
// unused candidate reads is never used.
struct ColWalkJob {
    const unsigned long long* key;
    const void* b_base;  // row i holds B_i, i = 0 .. k-1
    int32_t* score;
    int32_t* xs;
    int b_pitch, n_keys;
    int n, w, k;
};

template <int CAP>
struct ColWalkPack {
    ColWalkJob job[CAP];
    int count;
};

template <typename AT, int U1, int U2>
__device__ __forceinline__ bool colwalk_trip(const ColWalkJob& a, int lane, int& x, int& i) {
    const int n = a.n, w = a.w, k = a.k, D = 2 * n - 1;
    const AT* B = static_cast<const AT*>(a.b_base);
    const size_t pitch = (size_t)a.b_pitch;
    const int i1 = min(i + 1, k - 1), i2 = min(i + 2, k - 1);
    const int c0v = B[(size_t)i * pitch + (size_t)x];
    int c1[U1], c2[U2 > 0 ? U2 : 1];
#pragma unroll
    for (int u = 0; u < U1; ++u) {
        const int xc = min(max(x + lane + 64 * u - (n - 1), 0), w - 1);
        c1[u] = B[(size_t)i1 * pitch + (size_t)xc];
    }
#pragma unroll
    for (int u = 0; u < U2; ++u) {
        const int xc = min(max(x + lane + 64 * u - 2 * (n - 1), 0), w - 1);
        c2[u] = B[(size_t)i2 * pitch + (size_t)xc];
    }
    // no branch until every load of the trip has been used
    const int r0 = __builtin_amdgcn_readfirstlane(c0v);
    const int x1 = x + r0 - (n - 1);
    bool ok = r0 < D && (unsigned)x1 < (unsigned)w;
    int q = r0;  // candidate index of the second link's column: d_i + n - 1
    int m1 = c1[0];
#pragma unroll
    for (int u = 1; u < U1; ++u) m1 = (q >> 6) == u ? c1[u] : m1;
    const int r1 = __builtin_amdgcn_readlane(m1, q & 63);
    const int x2 = x1 + r1 - (n - 1);
    const bool two = i + 1 < k;
    const bool ok2 = ok && two && r1 < D && (unsigned)x2 < (unsigned)w;
    int r2 = 0, x3 = 0;
    bool ok3 = false;
    const bool three = U2 > 0 && i + 2 < k;
    if constexpr (U2 > 0) {
        const int q2 = r0 + r1;  // (x2 - x) + 2(n - 1)
        int m2 = c2[0];
#pragma unroll
        for (int u = 1; u < U2; ++u) m2 = (q2 >> 6) == u ? c2[u] : m2;
        r2 = __builtin_amdgcn_readlane(m2, q2 & 63);
        x3 = x2 + r2 - (n - 1);
        ok3 = ok2 && three && r2 < D && (unsigned)x3 < (unsigned)w;
    }
    if (lane == 0) {
        if (ok) a.xs[i + 1] = x1;
        if (ok2) a.xs[i + 2] = x2;
        if (ok3) a.xs[i + 3] = x3;
    }
    if (!ok || (two && !ok2) || (three && !ok3)) return false;
    if (three) {
        x = x3;
        i += 3;
    } else if (two) {
        x = x2;
        i += 2;
    } else {
        x = x1;
        i += 1;
    }
    return true;
}

template <typename AT, int CAP>
__global__ __launch_bounds__(64) void walk_colmax(ColWalkPack<CAP> pk) {
    const ColWalkJob& a = pk.job[blockIdx.x];
    const int lane = threadIdx.x;
    unsigned long long m = 0;
    for (int q0 = 0; q0 < a.n_keys; q0 += 64 * 8) {
        unsigned long long t[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int q = q0 + u * 64 + lane;
            t[u] = q < a.n_keys ? a.key[q] : 0ull;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) m = t[u] > m ? t[u] : m;
    }
    m = wave_max_u64(m);
    const unsigned int xu = 0xffffffffu - (unsigned int)(m & 0xffffffffull);
    if ((m >> 32) == 0 || xu >= (unsigned int)a.w) {
        if (lane == 0) *a.score = -1;
        return;
    }
    int x = (int)xu, i = 0;
    if (lane == 0) a.xs[0] = x;
    const int D = 2 * a.n - 1;
    while (i < a.k) {
        const bool ok = D <= 255    ? colwalk_trip<AT, 4, 8>(a, lane, x, i)
                        : D <= 511  ? colwalk_trip<AT, 8, 0>(a, lane, x, i)
                        : D <= 1023 ? colwalk_trip<AT, 16, 0>(a, lane, x, i)
                                    : colwalk_trip<AT, 32, 0>(a, lane, x, i);
        if (!ok) {
            if (lane == 0) *a.score = -1;
            return;
        }
    }
    if (lane == 0) *a.score = (int)(m >> 32) - 1;
}

// ---- host side ---------------------------------------------------------------

// Kernels of one step launch are chosen by this class; images of one class
// can share launches.
struct DpClass {
    int kind;   // WindowKind
    int bound;  // fixed kernels: the template bound
    int dc;     // fixed kernels: displacements per thread
    bool a16;
    bool narrow;  // uint16 tables (bands 0 .. k-2)
    int steps;    // most DP steps per launch allowed, 1..3 (tuning)
    int stripe;   // item-order stripe of the multi-step kernels (tuning)
    bool operator==(const DpClass& o) const {
        return kind == o.kind && bound == o.bound && dc == o.dc && a16 == o.a16 &&
               narrow == o.narrow && steps == o.steps && stripe == o.stripe;
    }
};

// Table of band i of an image (the last band is always int32: the DP reads
// it as V_{k-1}).
const void* band_table(const DpJobSpec& J, int i) {
    const size_t band = (size_t)J.g.D * J.g.W;
    if (i < J.tables.narrow) return J.tables.tab16 + (size_t)i * band;
    return J.tables.wide + (size_t)(i - J.tables.narrow) * band;
}

const int32_t* last_table(const DpJobSpec& J) {
    return static_cast<const int32_t*>(band_table(J, J.g.k - 1));
}

// The column recurrence takes unbounded bends without a through-point pin,
// k >= 2 and at least three displacements (its k rows of back-pointers fit
// in the space of the k-2 planes, or one, of D rows each).
bool colmax_apply(const DpJobSpec& J) {
    return J.plan.kind == WindowKind::Full && J.pin.j < 0 && J.g.k >= 2 && J.g.D >= 3;
}

DpClass class_of(const DpJobSpec& j) {
    DpClass c;
    c.kind = (int)j.plan.kind;
    const bool fixed = j.plan.kind == WindowKind::Fixed;
    c.bound = fixed ? j.plan.bound : 0;
    c.dc = fixed ? j.plan.dc : kDCGeneric;
    c.a16 = j.plan.a16;
    c.narrow = j.tables.narrow > 0;
    c.steps = j.plan.steps;
    c.stripe = j.plan.stripe;
    if (j.plan.kind == WindowKind::Full && colmax_apply(j))
        c.kind = (int)WindowKind::Full;  // the column recurrence
    else if (!fixed)
        c.kind = (int)WindowKind::Generic;  // one scanning kernel for every other kind
    return c;
}

// Kernel family of a class's single-step launches (for the timing brackets).
const char* step_family(const DpClass& c) {
    return c.kind == (int)WindowKind::Fixed ? "dp_step_fixed" : "dp_step_generic";
}

int items_y_of(const Geometry& g, int dc) {
    const int chunks = (g.D + dc - 1) / dc;
    return (chunks + kWaves - 1) / kWaves;
}

template <int B, typename AT, int CAP, typename TT>
void launch_fixed_b(int dc, hipStream_t s, const DpPack<CAP>& pk) {
    if (dc == 8)
        hipLaunchKernelGGL((dp_step_fixed<B, 8, AT, CAP, TT>), dim3(pk.total), dim3(64 * kWaves), 0,
                           s, pk);
    else
        hipLaunchKernelGGL((dp_step_fixed<B, 16, AT, CAP, TT>), dim3(pk.total), dim3(64 * kWaves),
                           0, s, pk);
}

template <typename AT, int CAP, typename TT>
hipError_t launch_step_t(const DpClass& c, hipStream_t s, const DpPack<CAP>& pk) {
    if (c.kind != (int)WindowKind::Fixed) {
        hipLaunchKernelGGL((dp_step_generic<AT, CAP, TT>), dim3(pk.total), dim3(64 * kWaves), 0, s,
                           pk);
        return hipSuccess;
    }
#define FHTP_B(BB) \
    case BB: launch_fixed_b<BB, AT, CAP, TT>(c.dc, s, pk); return hipSuccess;
    switch (c.bound) {
        FHTP_B(0) FHTP_B(1) FHTP_B(2) FHTP_B(3) FHTP_B(4) FHTP_B(5) FHTP_B(6) FHTP_B(7) FHTP_B(8)
        FHTP_B(9) FHTP_B(10) FHTP_B(11) FHTP_B(12) FHTP_B(13) FHTP_B(14) FHTP_B(15) FHTP_B(16)
        default: return hipErrorInvalidValue;
    }
#undef FHTP_B
}

template <typename AT, int CAP>
hipError_t launch_step(const DpClass& c, hipStream_t s, const DpPack<CAP>& pk) {
    return c.narrow ? launch_step_t<AT, CAP, uint16_t>(c, s, pk)
                    : launch_step_t<AT, CAP, int32_t>(c, s, pk);
}

// Pin on V_{k-1} read from the table H_{k-1}: x_{k-1} is the column of the
// cell, x_k its column plus its displacement.
void first_step_pin(const DpJobSpec& J, int& mode, int& x) {
    mode = J.pin.j == J.g.k - 1 ? 1 : J.pin.j == J.g.k ? 2 : 0;
    x = mode ? J.pin.x : 0;
}

// Common fields of an image's step descriptor.
DpJob base_job(const DpJobSpec& J) {
    const Geometry& g = J.g;
    DpJob a{};
    a.n = g.n;
    a.w = g.w;
    a.bound = J.plan.bound;
    a.full = J.plan.kind == WindowKind::Full;
    a.win = J.plan.kind == WindowKind::Angle ? J.buf.win : nullptr;
    a.h_pitch = g.W;
    a.v_pitch = g.pitch;
    a.a_pitch = g.pitch;
    a.items_x = (g.w + 63) / 64;
    a.out_pin_x = -1;
    return a;
}

// The block kernel takes scanned windows (the angle form, bounds above the
// fixed-window kernels') of bands with at most 255 displacements, without a
// through-point pin.
bool blocks_apply(const DpJobSpec& J) {
    return (J.plan.kind == WindowKind::Angle || J.plan.kind == WindowKind::Generic) &&
           J.pin.j < 0 && J.g.D <= kBlkRows - 1;
}

// Steps of a pack of images of one class (each with k >= 2).
template <typename AT, int CAP>
hipError_t run_steps(const DpClass& c, const std::vector<const DpJobSpec*>& jobs, hipStream_t s) {
    int max_steps = 0;
    for (const DpJobSpec* J : jobs) max_steps = std::max(max_steps, J->g.k - 1);
    // Steps that take the block kernel and the others, each run of launches
    // of one kernel in one timing bracket.
    auto blocks_at = [&](const DpJobSpec& J, int) { return blocks_apply(J); };
    std::vector<const char*> seq;  // kernel family of every launch, in order
    for (int st = 0; st < max_steps; ++st) {
        bool b = false, o = false;
        for (const DpJobSpec* J : jobs) {
            if (J->g.k - 1 <= st) continue;
            (blocks_at(*J, st) ? b : o) = true;
        }
        if (b) seq.push_back("dp_step_blocks");
        if (o) seq.push_back(step_family(c));
    }
    std::unique_ptr<TimedLaunch> tl;
    size_t q = 0;
    auto bracket = [&]() {  // before launch q: a bracket per run of one family
        if (q == 0 || seq[q] != seq[q - 1]) {
            tl.reset();
            size_t e = q;
            while (e < seq.size() && seq[e] == seq[q]) ++e;
            tl.reset(new TimedLaunch(seq[q], s, (int)(e - q)));
        }
        ++q;
    };
    for (int st = 0; st < max_steps; ++st) {
        DpPack<CAP> pk{}, pb{};
        long long total = 0, tb = 0;
        int cnt = 0, cb = 0;
        for (const DpJobSpec* J : jobs) {
            const Geometry& g = J->g;
            if (g.k - 1 <= st) continue;
            const int i = g.k - 2 - st;  // band of this step
            const size_t plane = (size_t)g.D * g.pitch;
            DpJob a = base_job(*J);
            a.vin = st == 0 ? last_table(*J)
                            : J->buf.vplanes + (size_t)((i + 1) & 1) * plane;
            a.vin_pitch = st == 0 ? g.W : g.pitch;
            a.htab = band_table(*J, i);
            const bool last = i == 0;
            // two planes in turn: step i only overwrites V_{i+2}, whose readers
            // (step i+1) finished with the previous launch
            a.vout = last ? nullptr : J->buf.vplanes + (size_t)(i & 1) * plane;
            a.aout = last ? nullptr : static_cast<AT*>(J->buf.a) + (size_t)(i - 1) * plane;
            a.key = last ? J->buf.key : nullptr;
            a.succ = last ? J->buf.succ : nullptr;
            if (st == 0) first_step_pin(*J, a.vin_pin, a.vin_pin_x);
            a.out_pin_x = J->pin.j == i ? J->pin.x : -1;
            if (blocks_at(*J, st)) {
                a.items_x = (g.w + kBlkCols - 1) / kBlkCols;
                a.items_y = 1;
                a.item0 = (int)tb;
                tb += a.items_x;
                if (tb > 0x7fffffffLL) return hipErrorInvalidConfiguration;
                pb.job[cb++] = a;
                continue;
            }
            a.items_y = items_y_of(g, c.dc);
            a.item0 = (int)total;
            total += (long long)a.items_x * a.items_y;
            if (total > 0x7fffffffLL) return hipErrorInvalidConfiguration;
            pk.job[cnt++] = a;
        }
        if (cb > 0) {
            pb.count = cb;
            pb.total = (int)tb;
            bracket();
            if (c.narrow)
                hipLaunchKernelGGL((dp_step_blocks<AT, CAP, uint16_t>), dim3((unsigned)tb),
                                   dim3(kBlkThreads), 0, s, pb);
            else
                hipLaunchKernelGGL((dp_step_blocks<AT, CAP, int32_t>), dim3((unsigned)tb),
                                   dim3(kBlkThreads), 0, s, pb);
            hipError_t e = hipGetLastError();
            if (e != hipSuccess) return e;
        }
        if (cnt > 0) {
            pk.count = cnt;
            pk.total = (int)total;
            bracket();
            hipError_t e = launch_step<AT, CAP>(c, s, pk);
            if (e != hipSuccess) return e;
        }
    }
    return hipSuccess;
}

template <typename AT, int CAP, bool PIN, typename TT>
hipError_t launch_pair_p(int bound, hipStream_t s, int grid, const DpPairPack<CAP>& pk) {
#define FHTP_B(BB)                                                                         \
    case BB:                                                                               \
        hipLaunchKernelGGL((dp_pair_fixed<BB, AT, CAP, PIN, TT>), dim3(grid),              \
                           dim3(64 * kPairWaves), 0, s, pk);                               \
        return hipSuccess;
    switch (bound) {
        FHTP_B(0) FHTP_B(1) FHTP_B(2) FHTP_B(3) FHTP_B(4) FHTP_B(5) FHTP_B(6) FHTP_B(7) FHTP_B(8)
        FHTP_B(9) FHTP_B(10) FHTP_B(11) FHTP_B(12) FHTP_B(13) FHTP_B(14) FHTP_B(15) FHTP_B(16)
        default: return hipErrorInvalidValue;
    }
#undef FHTP_B
}

// Pinned packs exist only for single images (a batch job has no pin).
template <typename AT, int CAP, typename TT>
hipError_t launch_pair_t(int bound, bool pinned, hipStream_t s, int grid,
                         const DpPairPack<CAP>& pk) {
    if constexpr (CAP == 1) {
        if (pinned) return launch_pair_p<AT, CAP, true, TT>(bound, s, grid, pk);
    } else {
        if (pinned) return hipErrorInvalidValue;
    }
    return launch_pair_p<AT, CAP, false, TT>(bound, s, grid, pk);
}

template <typename AT, int CAP>
hipError_t launch_pair(int bound, bool pinned, bool narrow, hipStream_t s, int grid,
                       const DpPairPack<CAP>& pk) {
    return narrow ? launch_pair_t<AT, CAP, uint16_t>(bound, pinned, s, grid, pk)
                  : launch_pair_t<AT, CAP, int32_t>(bound, pinned, s, grid, pk);
}

template <typename AT, int CAP, typename TT>
hipError_t launch_triple_t(int bound, hipStream_t s, int grid, const DpTriplePack<CAP>& pk) {
#define FHTP_B(BB)                                                                         \
    case BB:                                                                               \
        hipLaunchKernelGGL((dp_triple_fixed<BB, AT, CAP, TT>), dim3(grid),                 \
                           dim3(64 * kPairWaves), 0, s, pk);                               \
        return hipSuccess;
    switch (bound) {
        FHTP_B(0) FHTP_B(1) FHTP_B(2) FHTP_B(3) FHTP_B(4) FHTP_B(5) FHTP_B(6) FHTP_B(7) FHTP_B(8)
        default: return hipErrorInvalidValue;
    }
#undef FHTP_B
}

template <typename AT, int CAP>
hipError_t launch_triple(int bound, bool narrow, hipStream_t s, int grid,
                         const DpTriplePack<CAP>& pk) {
    return narrow ? launch_triple_t<AT, CAP, uint16_t>(bound, s, grid, pk)
                  : launch_triple_t<AT, CAP, int32_t>(bound, s, grid, pk);
}

// Two steps per launch need the fixed window, the 8-displacement chunk (an
// image whose step grid leaves the chip latency-bound on its own) and byte
// offsets inside a workgroup's rows that fit 32 bits.
bool pairs_apply(const DpJobSpec& J) {
    const Geometry& g = J.g;
    const long long rows = kPairRows + 4LL * kMaxFixedB + kStrip;  // the widest view
    const long long pitch = std::max(g.W, g.pitch);
    return J.plan.steps >= 2 && J.plan.kind == WindowKind::Fixed && J.plan.dc == kPairDC &&
           g.k >= 2 && rows * pitch * 4 < 0x7fffffffLL;
}

// Three steps per launch: as two, with a bound of at most kTriMaxB and no pin.
bool triples_apply(const DpJobSpec& J) {
    return pairs_apply(J) && J.plan.steps >= 3 && J.plan.bound <= kTriMaxB && J.pin.j < 0;
}

// Steps of a pack of images of one class with bands k-2 .. 1 taken G = 2 or
// 3 per launch, then the last step.  Images are aligned at the end: every
// image's last step is in the final launch and its groups in the launches
// just before it.  The P = k-2 bands before the last step make P / G groups;
// the P % G top bands left over go ahead of all groups: one band alone in a
// one-step launch, two (G = 3) as a pair in a two-step launch.  Per image,
// the launches that make V alternate between its two value planes so that
// V_1 lands in plane 1, where the last step reads it; a launch never writes
// the plane it reads, and an image that sits out a launch leaves its planes
// untouched.
template <typename AT, int CAP>
hipError_t run_steps_grouped(const DpClass& c, int G, const std::vector<const DpJobSpec*>& jobs,
                             hipStream_t s) {
    int Q = 0;  // group launches
    bool singles = false, head_pairs = false;
    for (const DpJobSpec* J : jobs) {
        const int P = J->g.k - 2;
        Q = std::max(Q, P / G);
        singles = singles || P % G == 1;
        head_pairs = head_pairs || P % G == 2;
    }
    // V-launches of an image: the head (if any), then its groups.
    auto vlaunches = [G](const DpJobSpec& J) {
        const int P = J.g.k - 2;
        return (P % G ? 1 : 0) + P / G;
    };
    // Input plane of V-launch j of an image (j = 0: the table H_{k-1}) and its
    // output plane.
    auto plane_of = [&](const DpJobSpec& J, int j) {
        const int m = vlaunches(J);
        return J.buf.vplanes + (size_t)(((m - 1 - j) & 1) ? 0 : 1) * ((size_t)J.g.D * J.g.pitch);
    };
    auto input_of = [&](const DpJobSpec& J, int j, const int32_t*& vin, int& pitch) {
        if (j == 0) {
            vin = last_table(J);
            pitch = J.g.W;
        } else {
            vin = plane_of(J, j - 1);
            pitch = J.g.pitch;
        }
    };
    if (singles) {
        DpPack<CAP> pk{};
        long long total = 0;
        int cnt = 0;
        for (const DpJobSpec* J : jobs) {
            const Geometry& g = J->g;
            if ((g.k - 2) % G != 1) continue;
            const int i = g.k - 2;  // its top band
            DpJob a = base_job(*J);
            input_of(*J, 0, a.vin, a.vin_pitch);
            first_step_pin(*J, a.vin_pin, a.vin_pin_x);
            a.out_pin_x = J->pin.j == i ? J->pin.x : -1;
            a.htab = band_table(*J, i);
            a.vout = plane_of(*J, 0);
            a.aout = static_cast<AT*>(J->buf.a) + (size_t)(i - 1) * ((size_t)g.D * g.pitch);
            a.items_y = items_y_of(g, c.dc);
            a.item0 = (int)total;
            total += (long long)a.items_x * a.items_y;
            if (total > 0x7fffffffLL) return hipErrorInvalidConfiguration;
            pk.job[cnt++] = a;
        }
        pk.count = cnt;
        pk.total = (int)total;
        TimedLaunch tl(step_family(c), s);
        hipError_t e = launch_step<AT, CAP>(c, s, pk);
        if (e != hipSuccess) return e;
    }
    // A pair launch: image J's pair with phase-1 band i, as its V-launch j.
    auto pair_job = [&](const DpJobSpec& J, int i, int j, DpPairJob& a) {
        const Geometry& g = J.g;
        const size_t plane = (size_t)g.D * g.pitch;
        AT* A = static_cast<AT*>(J.buf.a);
        a = DpPairJob{};
        input_of(J, j, a.vin, a.vin_pitch);
        if (j == 0) first_step_pin(J, a.vin_pin, a.vin_pin_x);  // vin is H_{k-1}
        a.pin1_x = J.pin.j == i ? J.pin.x : -1;
        a.pin0_x = J.pin.j == i - 1 ? J.pin.x : -1;
        a.h1 = band_table(J, i);
        a.h0 = band_table(J, i - 1);
        a.vout = plane_of(J, j);
        a.a = A + (size_t)(i - 2) * plane;  // planes i-2 and i-1: A_i with the links after
        a.h_pitch = g.W;
        a.v_pitch = g.pitch;
        a.a_pitch = g.pitch;
        a.n = g.n;
        a.w = g.w;
        a.items_x = (g.w + 63) / 64;
        a.items_y = (g.D + kPairRows - 1) / kPairRows;
    };
    auto launch_pairs = [&](DpPairPack<CAP>& pk, int cnt, long long total) {
        pk.count = cnt;
        pk.stripe = std::max(1, c.stripe);
        bool pinned = false;
        for (int q = 0; q < cnt; ++q)
            pinned = pinned || pk.job[q].vin_pin != 0 || pk.job[q].pin1_x >= 0 || pk.job[q].pin0_x >= 0;
        return launch_pair<AT, CAP>(jobs[0]->plan.bound, pinned, c.narrow, s, (int)total, pk);
    };
    if (head_pairs) {  // G = 3: two top bands left over
        DpPairPack<CAP> pk{};
        long long total = 0;
        int cnt = 0;
        for (const DpJobSpec* J : jobs) {
            if ((J->g.k - 2) % G != 2) continue;
            DpPairJob a;
            pair_job(*J, J->g.k - 2, 0, a);
            a.item0 = (int)total;
            total += (long long)a.items_x * a.items_y;
            if (total > 0x7fffffffLL) return hipErrorInvalidConfiguration;
            pk.job[cnt++] = a;
        }
        TimedLaunch tl("dp_pair_fixed", s);
        hipError_t e = launch_pairs(pk, cnt, total);
        if (e != hipSuccess) return e;
    }
    // one timing bracket around the whole run of group launches
    TimedLaunch tl_groups(Q > 0 ? (G == 3 ? "dp_triple_fixed" : "dp_pair_fixed") : nullptr, s, Q);
    for (int L = 0; L < Q; ++L) {
        long long total = 0;
        int cnt = 0;
        hipError_t e;
        if (G == 2) {
            DpPairPack<CAP> pk{};
            for (const DpJobSpec* J : jobs) {
                const int P = J->g.k - 2, np = P / 2, odd = P & 1;
                const int t = L - (Q - np);  // the image's pair index in this launch
                if (t < 0) continue;
                DpPairJob a;
                pair_job(*J, P - odd - 2 * t, odd + t, a);  // phase 2 makes the band below
                a.item0 = (int)total;
                total += (long long)a.items_x * a.items_y;
                if (total > 0x7fffffffLL) return hipErrorInvalidConfiguration;
                pk.job[cnt++] = a;
            }
            e = launch_pairs(pk, cnt, total);
        } else {
            DpTriplePack<CAP> pk{};
            for (const DpJobSpec* J : jobs) {
                const Geometry& g = J->g;
                const int P = g.k - 2, nt = P / 3, rem = P % 3;
                const int t = L - (Q - nt);  // the image's triple index in this launch
                if (t < 0) continue;
                const int i = P - rem - 3 * t - 2;  // level-0 band; levels 1, 2 make i+1, i+2
                const int j = (rem ? 1 : 0) + t;
                const size_t plane = (size_t)g.D * g.pitch;
                AT* A = static_cast<AT*>(J->buf.a);
                DpTripleJob a{};
                input_of(*J, j, a.vin, a.vin_pitch);
                a.h2 = band_table(*J, i + 2);
                a.h1 = band_table(*J, i + 1);
                a.h0 = band_table(*J, i);
                a.vout = plane_of(*J, j);
                a.a0 = A + (size_t)(i - 1) * plane;  // A_{i+1}
                a.a1 = A + (size_t)i * plane;        // A_{i+2}
                a.a2 = A + (size_t)(i + 1) * plane;  // A_{i+3}
                a.vin_pitch = j == 0 ? g.W : g.pitch;
                a.h_pitch = g.W;
                a.v_pitch = g.pitch;
                a.a_pitch = g.pitch;
                a.n = g.n;
                a.w = g.w;
                a.items_x = (g.w + 63) / 64;
                a.items_y = (g.D + kPairRows - 1) / kPairRows;
                a.item0 = (int)total;
                total += (long long)a.items_x * a.items_y;
                if (total > 0x7fffffffLL) return hipErrorInvalidConfiguration;
                pk.job[cnt++] = a;
            }
            pk.count = cnt;
            pk.stripe = std::max(1, c.stripe);
            e = launch_triple<AT, CAP>(jobs[0]->plan.bound, c.narrow, s, (int)total, pk);
        }
        if (e != hipSuccess) return e;
    }
    // last step of every image: V_1 (or the table H_1 when k = 2) to the keys
    DpPack<CAP> pk{};
    long long total = 0;
    int cnt = 0;
    for (const DpJobSpec* J : jobs) {
        const Geometry& g = J->g;
        const int m = vlaunches(*J);
        DpJob a = base_job(*J);
        input_of(*J, m, a.vin, a.vin_pitch);
        if (m == 0) first_step_pin(*J, a.vin_pin, a.vin_pin_x);  // k = 2: vin is H_1
        a.out_pin_x = J->pin.j == 0 ? J->pin.x : -1;
        a.htab = band_table(*J, 0);
        a.key = J->buf.key;
        a.succ = J->buf.succ;
        a.items_y = items_y_of(g, c.dc);
        a.item0 = (int)total;
        total += (long long)a.items_x * a.items_y;
        if (total > 0x7fffffffLL) return hipErrorInvalidConfiguration;
        pk.job[cnt++] = a;
    }
    pk.count = cnt;
    pk.total = (int)total;
    tl_groups.close();
    TimedLaunch tl(step_family(c), s);
    return launch_step<AT, CAP>(c, s, pk);
}

// Steps of the column recurrence for a pack of images: launch L makes band
// Q-1-L of every image with more bands than that (Q: the most bands), so
// every image's band 0 is in the final launch.  U_i goes to row 0 of value
// plane i & 1, B_i to row i of the back-pointer space.  An image's top band
// reads an int32 table and the others its narrow ones when it has them, so a
// launch splits into a pack of each where both occur.
template <typename AT, int CAP>
hipError_t run_colmax(const DpClass& c, const std::vector<const DpJobSpec*>& jobs, hipStream_t s) {
    int Q = 0;
    for (const DpJobSpec* J : jobs) Q = std::max(Q, J->g.k);
    TimedLaunch tl("dp_colmax", s, Q);
    for (int L = 0; L < Q; ++L) {
        const int i = Q - 1 - L;
        for (int wide = 1; wide >= 0; --wide) {
            ColPack<CAP> pk{};
            long long total = 0;
            int cnt = 0;
            for (const DpJobSpec* J : jobs) {
                const Geometry& g = J->g;
                if (g.k <= i) continue;
                const bool is_wide = i >= J->tables.narrow;
                if (is_wide != (wide == 1)) continue;
                const size_t plane = (size_t)g.D * g.pitch;
                ColJob a{};
                a.htab = band_table(*J, i);
                a.uin = i == g.k - 1 ? nullptr : J->buf.vplanes + (size_t)((i + 1) & 1) * plane;
                a.uout = i == 0 ? nullptr : J->buf.vplanes + (size_t)(i & 1) * plane;
                a.bout = static_cast<AT*>(J->buf.a) + (size_t)i * g.pitch;
                a.key = i == 0 ? J->buf.key : nullptr;
                a.h_pitch = g.W;
                a.n = g.n;
                a.w = g.w;
                a.item0 = (int)total;
                total += (g.w + 63) / 64;
                if (total > 0x7fffffffLL) return hipErrorInvalidConfiguration;
                pk.job[cnt++] = a;
            }
            if (cnt == 0) continue;
            pk.count = cnt;
            const dim3 grid((unsigned)total), block(64 * kColWaves);
            if (!wide && c.narrow)
                hipLaunchKernelGGL((dp_colmax<AT, CAP, uint16_t>), grid, block, 0, s, pk);
            else
                hipLaunchKernelGGL((dp_colmax<AT, CAP, int32_t>), grid, block, 0, s, pk);
            hipError_t e = hipGetLastError();
            if (e != hipSuccess) return e;
        }
    }
    return hipSuccess;
}

template <typename AT, int CAP>
hipError_t run_colmax_walks(const std::vector<const DpJobSpec*>& jobs, hipStream_t s) {
    for (size_t q0 = 0; q0 < jobs.size(); q0 += CAP) {
        ColWalkPack<CAP> pk{};
        const int cnt = (int)std::min<size_t>(CAP, jobs.size() - q0);
        for (int q = 0; q < cnt; ++q) {
            const DpJobSpec& J = *jobs[q0 + q];
            ColWalkJob& a = pk.job[q];
            a.key = J.buf.key;
            a.b_base = J.buf.a;
            a.score = J.score;
            a.xs = J.xs;
            a.b_pitch = J.g.pitch;
            a.n_keys = (J.g.w + 63) / 64;
            a.n = J.g.n;
            a.w = J.g.w;
            a.k = J.g.k;
        }
        pk.count = cnt;
        {
            TimedLaunch tl("walk_colmax", s);
            hipLaunchKernelGGL((walk_colmax<AT, CAP>), dim3(cnt), dim3(64), 0, s, pk);
        }
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template <typename AT, int CAP>
hipError_t run_walks(const std::vector<const DpJobSpec*>& jobs,
                     const std::vector<std::pair<const DpJobSpec*, int>>& grouped, hipStream_t s) {
    for (size_t q0 = 0; q0 < jobs.size(); q0 += CAP) {
        WalkPack<CAP> pk{};
        const int cnt = (int)std::min<size_t>(CAP, jobs.size() - q0);
        for (int q = 0; q < cnt; ++q) {
            const DpJobSpec& J = *jobs[q0 + q];
            const Geometry& g = J.g;
            const DpClass c = class_of(J);
            WalkJob& a = pk.job[q];
            a.key = J.buf.key;
            a.succ = J.buf.succ;
            a.n_keys = g.k == 1        ? (int)(((g.w + 63) / 64) * items_y_of(g, kDCGeneric))
                       : blocks_apply(J) ? (g.w + kBlkCols - 1) / kBlkCols  // one per column tile
                                         : (int)(((g.w + 63) / 64) * items_y_of(g, c.dc));
            a.a_base = J.buf.a;
            a.a_plane = (size_t)g.D * g.pitch;
            a.a_pitch = g.pitch;
            a.n = g.n;
            a.w = g.w;
            a.k = g.k;
            a.bound = J.plan.bound;
            a.full = J.plan.kind == WindowKind::Full;
            a.win = J.plan.kind == WindowKind::Angle ? J.buf.win : nullptr;
            a.score = J.score;
            a.xs = J.xs;
            // run_steps_grouped with G = 2 makes bands 1 .. P - (P & 1) in
            // pairs, P = k - 2; with G = 3 bands 1 .. 3(P / 3) in triples and,
            // when two bands are left over, those two as a pair
            int G = 1;
            for (const auto& e : grouped)
                if (e.first == &J) G = e.second;
            const int P = g.k - 2;
            a.tri_top = G == 3 ? 3 * (P / 3) : 0;
            a.pair_lo = G == 3 ? a.tri_top + 1 : 1;
            a.pair_top = G == 2 ? P - (P & 1) : G == 3 && P % 3 == 2 ? P : 0;
        }
        pk.count = cnt;
        {
            TimedLaunch tl("walk", s);
            hipLaunchKernelGGL((walk<AT, CAP>), dim3(cnt), dim3(64), 0, s, pk);
        }
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template <typename AT, int CAP>
hipError_t launch_dp_jobs_t(const std::vector<const DpJobSpec*>& jobs, hipStream_t s) {
    // k = 1: the argmax of H_0, in packs.
    std::vector<const DpJobSpec*> single;
    for (const DpJobSpec* J : jobs)
        if (J->g.k == 1) single.push_back(J);
    for (size_t q0 = 0; q0 < single.size(); q0 += CAP) {
        DpPack<CAP> pk{};
        long long total = 0;
        const int cnt = (int)std::min<size_t>(CAP, single.size() - q0);
        for (int q = 0; q < cnt; ++q) {
            const DpJobSpec& J = *single[q0 + q];
            DpJob a = base_job(J);
            a.htab = band_table(J, 0);  // k = 1: the only band is int32
            a.key = J.buf.key;
            a.succ = J.buf.succ;
            first_step_pin(J, a.vin_pin, a.vin_pin_x);
            a.items_y = items_y_of(J.g, kDCGeneric);
            a.item0 = (int)total;
            total += (long long)a.items_x * a.items_y;
            if (total > 0x7fffffffLL) return hipErrorInvalidConfiguration;
            pk.job[q] = a;
        }
        pk.count = cnt;
        pk.total = (int)total;
        TimedLaunch tl("argmax_table", s);
        hipLaunchKernelGGL((argmax_table<CAP>), dim3(pk.total), dim3(64 * kWaves), 0, s, pk);
    }
    // k >= 2: step launches per class, in packs.
    std::vector<const DpJobSpec*> rest;
    for (const DpJobSpec* J : jobs)
        if (J->g.k >= 2) rest.push_back(J);
    std::vector<bool> done(rest.size(), false);
    std::vector<std::pair<const DpJobSpec*, int>> grouped;  // images whose steps went G per launch
    std::vector<const DpJobSpec*> colmax, walked;  // the column recurrence, the others
    for (size_t q = 0; q < rest.size(); ++q) {
        if (done[q]) continue;
        const DpClass c = class_of(*rest[q]);
        std::vector<const DpJobSpec*> group;
        for (size_t r = q; r < rest.size(); ++r)
            if (!done[r] && class_of(*rest[r]) == c) {
                group.push_back(rest[r]);
                done[r] = true;
            }
        for (size_t q0 = 0; q0 < group.size(); q0 += CAP) {
            std::vector<const DpJobSpec*> pack(group.begin() + q0,
                                               group.begin() + std::min(group.size(), q0 + CAP));
            if (c.kind == (int)WindowKind::Full) {
                hipError_t e = run_colmax<AT, CAP>(c, pack, s);
                if (e != hipSuccess) return e;
                colmax.insert(colmax.end(), pack.begin(), pack.end());
                continue;
            }
            // G steps per launch when every image qualifies and one has a
            // group of G steps
            bool all2 = true, all3 = true;
            int kmax = 0;
            for (const DpJobSpec* J : pack) {
                all2 = all2 && pairs_apply(*J) && (CAP == 1 || J->pin.j < 0);
                all3 = all3 && triples_apply(*J);
                kmax = std::max(kmax, J->g.k);
            }
            const int G = all3 && kmax >= 5 ? 3 : all2 && kmax >= 4 ? 2 : 1;
            hipError_t e = G > 1 ? run_steps_grouped<AT, CAP>(c, G, pack, s)
                                 : run_steps<AT, CAP>(c, pack, s);
            if (e != hipSuccess) return e;
            if (G > 1)
                for (const DpJobSpec* J : pack) grouped.emplace_back(J, G);
        }
    }
    for (const DpJobSpec* J : jobs)
        if (std::find(colmax.begin(), colmax.end(), J) == colmax.end()) walked.push_back(J);
    if (!colmax.empty()) {
        hipError_t e = run_colmax_walks<AT, CAP>(colmax, s);
        if (e != hipSuccess) return e;
    }
    return run_walks<AT, CAP>(walked, grouped, s);
}

}  // namespace

size_t dp_plane_bytes(const Geometry& g) { return (size_t)g.D * g.pitch * sizeof(int32_t); }

size_t dp_key_count(const Geometry& g) {
    // workgroups of the last step: at 8 displacements per thread (the
    // largest grid of the 64-column kernels), or one per column tile of the
    // block kernel
    const size_t k64 = (size_t)((g.w + 63) / 64) * items_y_of(g, 8);
    const size_t k16 = (size_t)((g.w + kBlkCols - 1) / kBlkCols);
    return k64 > k16 ? k64 : k16;
}

size_t dp_backptr_bytes(const Geometry& g, bool a16) {
    // Planes for A_2 .. A_{k-1}; there is no A_1 plane: the last step records,
    // with each workgroup's key, the successor of that cell (its row in the
    // succ buffer), and the walk starts from it.
    const size_t planes = g.k > 2 ? (size_t)(g.k - 2) : 1;
    return planes * g.D * g.pitch * (a16 ? 2 : 1);
}

hipError_t launch_dp_jobs(const DpJobSpec* jobs, int count, hipStream_t s) {
    std::vector<const DpJobSpec*> a8, a16;
    for (int q = 0; q < count; ++q) {
        const DpJobSpec& J = jobs[q];
        if (J.plan.kind == WindowKind::Fixed &&
            (J.plan.bound < 0 || J.plan.bound > kMaxFixedB || (J.plan.dc != 8 && J.plan.dc != 16)))
            return hipErrorInvalidValue;
        if (J.plan.kind == WindowKind::Angle) {
            TimedLaunch tl("angle_windows", s);
            hipLaunchKernelGGL(angle_windows, dim3(J.g.D), dim3(64), 0, s, J.g.n,
                               J.plan.tan_gamma, J.buf.win);
        }
        (J.plan.a16 ? a16 : a8).push_back(&J);
    }
    hipError_t e = hipSuccess;
    if (count == 1) {
        e = a8.empty() ? launch_dp_jobs_t<uint16_t, 1>(a16, s) : launch_dp_jobs_t<uint8_t, 1>(a8, s);
    } else {
        if (!a8.empty()) e = launch_dp_jobs_t<uint8_t, kPack>(a8, s);
        if (e == hipSuccess && !a16.empty()) e = launch_dp_jobs_t<uint16_t, kPack>(a16, s);
    }
    if (e != hipSuccess) return e;
    return hipGetLastError();
}

hipError_t launch_dp(const TableSet& tables, const Geometry& g, const DpPlan& plan,
                     const DpBuffers& buf, int32_t* score, int32_t* xs, hipStream_t stream,
                     Pin pin) {
    DpJobSpec j{tables, g, plan, buf, score, xs, pin};
    return launch_dp_jobs(&j, 1, stream);
}

}  // namespace fhtp
