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
// The last step (i = 0) writes no plane: each workgroup reduces its cells to a
// packed key ((V + 1) << 32 | ~(x*D + r)) whose maximum is the best score with
// the smallest (x, d) on ties, and merges it with one 64-bit atomic max.  A
// single thread then follows the back-pointers (k-1 dependent loads).
#include "fhtp_internal.h"

namespace fhtp {
namespace {

constexpr int kDC = 16;        // displacements per thread
constexpr int kWaves = 4;      // waves per workgroup, one displacement chunk each
constexpr int kMaxFixedB = 16; // largest bend bound with a register-window kernel

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

// Block-wide max of v, merged into *key by thread 0.
__device__ __forceinline__ void block_key_max(unsigned long long v, unsigned long long* key) {
    __shared__ unsigned long long part[kWaves];
    v = wave_max_u64(v);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) part[wave] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long m = part[0];
#pragma unroll
        for (int q = 1; q < kWaves; ++q) m = part[q] > m ? part[q] : m;
        atomicMax(key, m);
    }
}

// V_{i+1}(x', d') with the feasibility mask: zero-based row r' = d' + n - 1.
__device__ __forceinline__ int load_v(const int32_t* __restrict__ vin, int pitch, int xp, int dp,
                                      int n, int w) {
    const int r = dp + n - 1;
    const bool ok = xp < w && r >= 0 && r < 2 * n - 1 && xp + dp >= 0 && xp + dp < w;
    return ok ? vin[(size_t)r * pitch + xp] : -1;
}

// Shared tail of every step kernel: one output cell (x' = xp, displacement d)
// with range maximum m reached at row ra.
template <typename AT>
__device__ __forceinline__ void emit(int m, int ra, int xp, int d, int n, int w,
                                     const int32_t* __restrict__ htab, int h_pitch,
                                     int32_t* __restrict__ vout, int v_pitch, AT* __restrict__ aout,
                                     int a_pitch, bool last, unsigned long long& best) {
    const int D = 2 * n - 1;
    const int r = d + n - 1;
    if (xp >= w || r >= D) return;
    aout[(size_t)r * a_pitch + xp] = (AT)(ra < 0 ? 0 : ra);
    const int x = xp - d;
    if (x < 0 || x >= w) return;
    const int val = m >= 0 ? htab[(size_t)r * h_pitch + x] + m : -1;
    if (last) {
        const unsigned long long kk = pack_key(val, x, r, D);
        best = kk > best ? kk : best;
    } else {
        vout[(size_t)r * v_pitch + x] = val;
    }
}

// Step with the mode-0 window [d - B, d + B] fixed at compile time.
template <int B, typename AT>
__global__ __launch_bounds__(64 * kWaves) void dp_step_fixed(
    const int32_t* __restrict__ vin, int vin_pitch, const int32_t* __restrict__ htab, int h_pitch,
    int32_t* __restrict__ vout, int v_pitch, AT* __restrict__ aout, int a_pitch,
    unsigned long long* __restrict__ key, int n, int w) {
    constexpr int L = 2 * B + 1;
    constexpr int NV = kDC + 2 * B;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int xp = blockIdx.x * 64 + lane;
    const int chunk = blockIdx.y * kWaves + wave;
    const int d0 = -(n - 1) + chunk * kDC;
    const bool last = key != nullptr;

    int v[NV];
#pragma unroll
    for (int j = 0; j < NV; ++j) v[j] = load_v(vin, vin_pitch, xp, d0 - B + j, n, w);

    // Suffix maxima inside window-length blocks (smallest index on ties).
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
    unsigned long long best = 0;
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
            const int m = s_wins ? sv[j] : pv;
            const int ia = s_wins ? si[j] : pi;
            const int ra = chunk * kDC - B + ia;  // row of d' = d0 - B + ia
            emit<AT>(m, ra, xp, d0 + j, n, w, htab, h_pitch, vout, v_pitch, aout, a_pitch, last,
                     best);
        }
    }
    if (last) block_key_max(best, key);
}

// Step with per-displacement windows [lo(d), hi(d)] (large mode-0 bounds and
// the angle form), scanning each window.
template <typename AT>
__global__ __launch_bounds__(64 * kWaves) void dp_step_generic(
    const int32_t* __restrict__ vin, int vin_pitch, const int32_t* __restrict__ htab, int h_pitch,
    int32_t* __restrict__ vout, int v_pitch, AT* __restrict__ aout, int a_pitch,
    unsigned long long* __restrict__ key, int n, int w, int bound,
    const int32_t* __restrict__ win) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int xp = blockIdx.x * 64 + lane;
    const int chunk = blockIdx.y * kWaves + wave;
    const int d0 = -(n - 1) + chunk * kDC;
    const int D = 2 * n - 1;
    const bool last = key != nullptr;
    unsigned long long best = 0;
    for (int j = 0; j < kDC; ++j) {
        const int d = d0 + j;
        const int r = d + n - 1;
        if (r >= D) break;
        int lo, hi;
        if (win) {
            lo = win[r];
            hi = win[D + r];
        } else {
            lo = max(d - bound, -(n - 1));
            hi = min(d + bound, n - 1);
        }
        int m = load_v(vin, vin_pitch, xp, lo, n, w);
        int ia = lo;
        for (int dp = lo + 1; dp <= hi; ++dp) {
            const int vv = load_v(vin, vin_pitch, xp, dp, n, w);
            if (vv > m) {
                m = vv;
                ia = dp;
            }
        }
        emit<AT>(m, ia + n - 1, xp, d, n, w, htab, h_pitch, vout, v_pitch, aout, a_pitch, last,
                 best);
    }
    if (last) block_key_max(best, key);
}

// Step without a bend limit (Section 2.2): every d shares the column maximum.
template <typename AT>
__global__ __launch_bounds__(64 * kWaves) void dp_step_full(
    const int32_t* __restrict__ vin, int vin_pitch, const int32_t* __restrict__ htab, int h_pitch,
    int32_t* __restrict__ vout, int v_pitch, AT* __restrict__ aout, int a_pitch,
    unsigned long long* __restrict__ key, int n, int w) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int xp = blockIdx.x * 64 + lane;
    const int chunk = blockIdx.y * kWaves + wave;
    const int d0 = -(n - 1) + chunk * kDC;
    const bool last = key != nullptr;
    int m = load_v(vin, vin_pitch, xp, -(n - 1), n, w);
    int ia = -(n - 1);
    for (int dp = -(n - 1) + 1; dp <= n - 1; ++dp) {
        const int vv = load_v(vin, vin_pitch, xp, dp, n, w);
        if (vv > m) {
            m = vv;
            ia = dp;
        }
    }
    unsigned long long best = 0;
    for (int j = 0; j < kDC; ++j)
        emit<AT>(m, ia + n - 1, xp, d0 + j, n, w, htab, h_pitch, vout, v_pitch, aout, a_pitch,
                 last, best);
    if (last) block_key_max(best, key);
}

// k = 1: the answer is the best masked cell of H_0.
__global__ __launch_bounds__(64 * kWaves) void argmax_table(const int32_t* __restrict__ htab,
                                                            int h_pitch, int n, int w,
                                                            unsigned long long* __restrict__ key) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int x = blockIdx.x * 64 + lane;
    const int chunk = blockIdx.y * kWaves + wave;
    const int D = 2 * n - 1;
    unsigned long long best = 0;
    for (int j = 0; j < kDC; ++j) {
        const int r = chunk * kDC + j;
        const int d = r - (n - 1);
        if (r >= D || x >= w || x + d < 0 || x + d >= w) continue;
        const unsigned long long kk = pack_key(htab[(size_t)r * h_pitch + x], x, r, D);
        best = kk > best ? kk : best;
    }
    block_key_max(best, key);
}

// Mode-1 windows: lo(d) and hi(d) bracket every d' with n*|d'-d| <= t*(n*n + d*d').
__global__ void angle_windows(int n, double t, int32_t* __restrict__ win) {
    const int D = 2 * n - 1;
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= D) return;
    const int d = r - (n - 1);
    int lo = n, hi = -n;
    for (int dp = -(n - 1); dp <= n - 1; ++dp) {
        const double lhs = (double)n * (double)abs(dp - d);
        const double rhs = t * ((double)n * (double)n + (double)d * (double)dp);
        if (lhs <= rhs) {
            if (lo == n) lo = dp;
            hi = dp;
        }
    }
    win[r] = lo;
    win[D + r] = hi;
}

__global__ void clear_key(unsigned long long* key) { *key = 0ull; }

// Follows the back-pointers from the best cell of V_0 (eq. (5)).  Indices are
// range-checked, so a corrupt key or plane ends the walk with score -1 rather
// than an out-of-bounds read.
template <typename AT>
__global__ void backtrace(const unsigned long long* __restrict__ key, const AT* __restrict__ a,
                          size_t a_plane, int a_pitch, int n, int w, int k,
                          int32_t* __restrict__ score, int32_t* __restrict__ xs) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const int D = 2 * n - 1;
    const unsigned long long kv = *key;
    const unsigned int lin = 0xffffffffu - (unsigned int)(kv & 0xffffffffull);
    const unsigned int xu = lin / (unsigned int)D;
    int x = (int)xu;
    int r = (int)(lin % (unsigned int)D);
    if ((kv >> 32) == 0 || xu >= (unsigned int)w) {
        *score = -1;
        return;
    }
    xs[0] = x;
    for (int i = 0; i + 1 < k; ++i) {
        const int x1 = x + r - (n - 1);
        if (x1 < 0 || x1 >= w) {
            *score = -1;
            return;
        }
        xs[i + 1] = x1;
        r = a[(size_t)i * a_plane + (size_t)r * a_pitch + x1];
        if (r >= D) {
            *score = -1;
            return;
        }
        x = x1;
    }
    xs[k] = x + r - (n - 1);
    *score = (int)(kv >> 32) - 1;
}

template <int B, typename AT>
hipError_t launch_fixed_b(dim3 grid, hipStream_t s, const int32_t* vin, int vp, const int32_t* h,
                          int hp, int32_t* vout, int op, AT* a, int ap,
                          unsigned long long* key, int n, int w) {
    hipLaunchKernelGGL((dp_step_fixed<B, AT>), grid, dim3(64 * kWaves), 0, s, vin, vp, h, hp,
                       vout, op, a, ap, key, n, w);
    return hipSuccess;
}

template <typename AT>
hipError_t launch_step(const DpPlan& plan, dim3 grid, hipStream_t s, const int32_t* vin, int vp,
                       const int32_t* h, int hp, int32_t* vout, int op, AT* a, int ap,
                       unsigned long long* key, int n, int w, const int32_t* win) {
    switch (plan.kind) {
        case WindowKind::Full:
            hipLaunchKernelGGL((dp_step_full<AT>), grid, dim3(64 * kWaves), 0, s, vin, vp, h, hp,
                               vout, op, a, ap, key, n, w);
            return hipSuccess;
        case WindowKind::Generic:
        case WindowKind::Angle:
            hipLaunchKernelGGL((dp_step_generic<AT>), grid, dim3(64 * kWaves), 0, s, vin, vp, h,
                               hp, vout, op, a, ap, key, n, w, plan.bound,
                               plan.kind == WindowKind::Angle ? win : nullptr);
            return hipSuccess;
        case WindowKind::Fixed:
            break;
    }
#define FHTP_B(BB) \
    case BB: return launch_fixed_b<BB, AT>(grid, s, vin, vp, h, hp, vout, op, a, ap, key, n, w);
    switch (plan.bound) {
        FHTP_B(0) FHTP_B(1) FHTP_B(2) FHTP_B(3) FHTP_B(4) FHTP_B(5) FHTP_B(6) FHTP_B(7) FHTP_B(8)
        FHTP_B(9) FHTP_B(10) FHTP_B(11) FHTP_B(12) FHTP_B(13) FHTP_B(14) FHTP_B(15) FHTP_B(16)
        default: return hipErrorInvalidValue;
    }
#undef FHTP_B
}

template <typename AT>
hipError_t launch_dp_t(const int32_t* tables, const Geometry& g, const DpPlan& plan,
                       const DpBuffers& buf, int32_t* score, int32_t* xs, hipStream_t s) {
    const int n = g.n, w = g.w, k = g.k, D = g.D;
    const size_t band_stride = (size_t)D * g.W;
    const int chunks = (D + kDC - 1) / kDC;
    dim3 grid((w + 63) / 64, (chunks + kWaves - 1) / kWaves, 1);
    AT* a = static_cast<AT*>(buf.a);
    const size_t a_plane = (size_t)D * g.pitch;

    hipLaunchKernelGGL(clear_key, dim3(1), dim3(1), 0, s, buf.key);
    if (plan.kind == WindowKind::Angle)
        hipLaunchKernelGGL(angle_windows, dim3((D + 255) / 256), dim3(256), 0, s, n,
                           plan.tan_gamma, buf.win);
    if (k == 1) {
        hipLaunchKernelGGL(argmax_table, grid, dim3(64 * kWaves), 0, s, tables, g.W, n, w,
                           buf.key);
    } else {
        const int32_t* vin = tables + (size_t)(k - 1) * band_stride;
        int vin_pitch = g.W;
        for (int i = k - 2; i >= 0; --i) {
            const bool last = i == 0;
            int32_t* vout = last ? nullptr : buf.v[i & 1];
            hipError_t e = launch_step<AT>(plan, grid, s, vin, vin_pitch,
                                           tables + (size_t)i * band_stride, g.W, vout, g.pitch,
                                           a + (size_t)i * a_plane, g.pitch,
                                           last ? buf.key : nullptr, n, w, buf.win);
            if (e != hipSuccess) return e;
            vin = vout;
            vin_pitch = g.pitch;
        }
    }
    hipLaunchKernelGGL((backtrace<AT>), dim3(1), dim3(64), 0, s, buf.key, a, a_plane, g.pitch, n,
                       w, k, score, xs);
    return hipGetLastError();
}

}  // namespace

size_t dp_plane_bytes(const Geometry& g) { return (size_t)g.D * g.pitch * sizeof(int32_t); }

size_t dp_backptr_bytes(const Geometry& g, bool a16) {
    const size_t planes = g.k > 1 ? (size_t)(g.k - 1) : 1;
    return planes * g.D * g.pitch * (a16 ? 2 : 1);
}

hipError_t launch_dp(const int32_t* tables, const Geometry& g, const DpPlan& plan,
                     const DpBuffers& buf, int32_t* score, int32_t* xs, hipStream_t stream) {
    if (plan.kind == WindowKind::Fixed && (plan.bound < 0 || plan.bound > kMaxFixedB))
        return hipErrorInvalidValue;
    if (plan.a16) return launch_dp_t<uint16_t>(tables, g, plan, buf, score, xs, stream);
    return launch_dp_t<uint8_t>(tables, g, plan, buf, score, xs, stream);
}

}  // namespace fhtp
