// Whole detections of small images in one launch: the band line sums
// (Section 2.1, eq. (1)), every DP step with its bend window (Sections
// 2.2-2.3, eqs. (3)-(4) and (6)-(7)), the global choice (main problem, steps
// 2-3) and the backtrace (eq. (5)), one workgroup per image with everything
// in LDS.
//
// For an image whose bands are at most 32 rows high and whose tables, value
// planes and back-pointers fit in 64 KB, the general path's launches (the
// FHT, one per one or two DP steps, the walk) are each a few microseconds of
// launch latency around very little work.  Here a workgroup loads the image
// into LDS once, then runs band by band from the bottom: the line sums H_i(x, d)
// for the cells the DP uses (x in [0, w), x + d in [0, w)) summed along the
// dyadic line (pixel by pixel for bands of up to 4 rows, from sums over blocks
// of 4 rows for taller ones), then the DP step on the previous band's values
// in LDS.  Line sums are exact integers, so any grouping of a line's pixels
// gives the same value as the stage recursion.  The dyadic offsets come from the
// recursive definition: the upper half of the line with shift s over n rows
// is the line with shift floor(s/2) over n/2 rows, the lower half the same
// line moved right by ceil(s/2); left-leaning lines mirror it.  Unrolled over
// the rows, the offset of row y is the sum, over the set bits l-1 of y, of
// ceil(s_l / 2), s_l being the shift at level l: a handful of scalar adds per
// line, since a wave's lanes share the shift.  Window maxima
// are scanned in ascending row order (ties to the smallest d'), the keys pick
// the largest value with the smallest (x, d), and the walk follows the
// back-pointers held in LDS: the same result as the general path, bit for
// bit.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <mutex>
#include <vector>

#include "fhtp_internal.h"

namespace fhtp {
namespace {

constexpr int kSmallThreads = 1024;  // 16 waves on the workgroup's CU
constexpr int kSmallMaxN = 32;
constexpr size_t kSmallLds = 64 * 1024;
constexpr int kSmallPack = 256;  // images per launch

struct SmallJob {
    const void* img;
    int32_t* score;
    int32_t* xs;
    int h, w, k, n;
    int kind;      // WindowKind
    int bound;     // mode-0 bound
    double tan_g;  // mode 1
};

template <int CAP>
struct SmallPack {
    SmallJob job[CAP];
    int count;
};

__host__ __device__ inline size_t align4(size_t b) { return (b + 3) & ~size_t(3); }

// LDS bytes of one image: its pixels, a band's line sums and two value
// planes, the back-pointers of every step, windows.
size_t small_lds_bytes(int n, int w, int k, int bpp) {
    const size_t D = 2 * (size_t)n - 1;
    return (kSmallThreads / 64) * 8 + align4((size_t)n * k * w * bpp) + 3 * D * w * 4 +
           align4((size_t)(k > 1 ? k - 1 : 0) * D * w) + 2 * D * 4;
}

__device__ __forceinline__ unsigned long long small_key(int val, int x, int r, int D) {
    const unsigned int lin = (unsigned int)x * (unsigned int)D + (unsigned int)r;
    return ((unsigned long long)(unsigned int)(val + 1) << 32) |
           (unsigned long long)(0xffffffffu - lin);
}

// N: the band height (a compile-time constant, so that a line's N reads are
// unrolled and in flight together).
template <typename PixT, int N, int CAP>
__global__ __launch_bounds__(kSmallThreads) void detect_small(SmallPack<CAP> pk) {
    extern __shared__ unsigned long long small_lds[];
    const SmallJob& a = pk.job[blockIdx.x];
    constexpr int n = N, D = 2 * N - 1;
    const int w = a.w, k = a.k;
    const int t = threadIdx.x;
    const int cells = D * w;
    constexpr int kRowLanes = kSmallThreads / 64;
    constexpr int kRowsPer = (D + kRowLanes - 1) / kRowLanes;  // rows per row lane
    // column lane, and row lane (uniform across a wave: its rows, shifts and
    // windows live in scalar registers)
    const int cx = t & 63, ry = __builtin_amdgcn_readfirstlane(t >> 6);
    unsigned long long* part = small_lds;  // one key per wave
    char* base = reinterpret_cast<char*>(small_lds + kSmallThreads / 64);
    PixT* img = reinterpret_cast<PixT*>(base);  // the whole image
    base += align4((size_t)n * k * w * sizeof(PixT));
    int* H = reinterpret_cast<int*>(base);
    int* Vp = H + cells;      // values of the band below (V_{i+1})
    int* Vc = Vp + cells;     // values of this band (V_i)
    unsigned char* A = reinterpret_cast<unsigned char*>(Vc + cells);  // A[i][r][x']
    base = reinterpret_cast<char*>(A) + align4((size_t)(k > 1 ? k - 1 : 0) * cells);
    int* wlo = reinterpret_cast<int*>(base);
    int* whi = wlo + D;

    // the image, once: 16-byte loads when the source is aligned, four in
    // flight per thread, then the bytes left over
    {
        const int bytes = n * k * w * (int)sizeof(PixT);
        const char* src = static_cast<const char*>(a.img);
        char* dst = reinterpret_cast<char*>(img);
        int done = 0;
        if ((reinterpret_cast<uintptr_t>(src) & 15) == 0) {
            const int n16 = bytes / 16;
            const uint4* s16 = reinterpret_cast<const uint4*>(src);
            uint4* d16 = reinterpret_cast<uint4*>(dst);
            for (int q0 = t; q0 < n16; q0 += 4 * kSmallThreads) {
                uint4 v[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int q = q0 + u * kSmallThreads;
                    v[u] = s16[q < n16 ? q : 0];
                }
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int q = q0 + u * kSmallThreads;
                    if (q < n16) d16[q] = v[u];
                }
            }
            done = n16 * 16;
        }
        for (int q0 = done + t; q0 < bytes; q0 += 4 * kSmallThreads) {
            char v[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int q = q0 + u * kSmallThreads;
                v[u] = src[q < bytes ? q : 0];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int q = q0 + u * kSmallThreads;
                if (q < bytes) dst[q] = v[u];
            }
        }
    }
    // windows [lo, hi] of every displacement, as rows
    for (int r = t; r < D; r += kSmallThreads) {
        const int d = r - (n - 1);
        int lo, hi;
        if (a.kind == (int)WindowKind::Angle) {
            lo = D;
            hi = -1;
            for (int rp = 0; rp < D; ++rp) {
                const int dp = rp - (n - 1);
                const double lhs = (double)n * (double)abs(dp - d);
                const double rhs = a.tan_g * ((double)n * (double)n + (double)d * (double)dp);
                if (lhs <= rhs) {
                    lo = min(lo, rp);
                    hi = max(hi, rp);
                }
            }
        } else if (a.kind == (int)WindowKind::Full) {
            lo = 0;
            hi = D - 1;
        } else {
            lo = max(d - a.bound, -(n - 1)) + n - 1;
            hi = min(d + a.bound, n - 1) + n - 1;
        }
        wlo[r] = lo;
        whi[r] = hi;
    }

    __syncthreads();
    // the windows of the thread's rows ry, ry + kRowLanes, ...
    int wl[kRowsPer], wh[kRowsPer];
#pragma unroll
    for (int q = 0; q < kRowsPer; ++q) {
        const int r = ry + q * kRowLanes;
        wl[q] = r < D ? wlo[r] : 0;
        wh[q] = r < D ? whi[r] : -1;
    }
    constexpr int p = N >= 32 ? 5 : N >= 16 ? 4 : N >= 8 ? 3 : N >= 4 ? 2 : N >= 2 ? 1 : 0;
    unsigned long long best = 0;
    for (int i = k - 1; i >= 0; --i) {
        const PixT* pix = img + (size_t)i * n * w;  // the band's pixels
        // line sums of the cells the DP uses; lanes along x, waves along the
        // rows (a row's shift, its offsets and y * w are uniform)
        if constexpr (N >= 8) {
            // Two levels of the recursion.  Every line of shift s crosses each
            // block of 4 rows along the 4-row line of shift s2 = s >> (p - 2)
            // (the levels below 4 rows see only the top bits of s), starting
            // at the line's offset on the block's first row.  So the sums of
            // the 4-row lines come first, per block m, shift s2 and direction
            // (j < 4: right-leaning s2 = j; j >= 4: left-leaning s2 = j - 3;
            // shift 0 is shared), in the plane of this band's values, which is
            // free until the DP step: 7n/4 * w ints, within its (2n-1) * w.
            constexpr int NB4 = N / 4;
            int* P = Vc;
            for (int x = cx; x < w; x += 64) {
                for (int cq = ry; cq < NB4 * 7; cq += kRowLanes) {
                    const int m = cq / 7, j = cq - m * 7;
                    const bool right = j < 4;
                    const int s2 = right ? j : j - 3;
                    const int o1 = ((s2 >> 1) + 1) >> 1, o2 = (s2 + 1) >> 1;  // rows 1, 2
                    const PixT* row = pix + (size_t)(4 * m) * w;
                    // columns clamped into the band: such sums are never used
                    auto px = [&](int t, int o) {
                        const int xx = min(max(right ? x + o : x - o, 0), w - 1);
                        return (int)row[t * w + xx];
                    };
                    P[cq * w + x] = px(0, 0) + px(1, o1) + px(2, o2) + px(3, o1 + o2);
                }
            }
            __syncthreads();
            for (int x = cx; x < w; x += 64) {
#pragma unroll
                for (int q = 0; q < kRowsPer; ++q) {
                    const int r = ry + q * kRowLanes;
                    if (r >= D) break;
                    const int d = r - (n - 1);
                    const int s = d < 0 ? -d : d;
                    const int s2 = s >> (p - 2);
                    const int j = d >= 0 ? s2 : (s2 == 0 ? 0 : 3 + s2);
                    // c[l] = ceil(s_l / 2), s_l = s >> (p - l), for the levels
                    // above 4 rows: the offset of block m's first row is the sum
                    // of c[l] over the set bits l-3 of m
                    int c[p + 1];
#pragma unroll
                    for (int l = 3; l <= p; ++l) c[l] = ((s >> (p - l)) + 1) >> 1;
                    int sum = 0;
                    if ((unsigned)(x + d) < (unsigned)w) {
#pragma unroll
                        for (int m = 0; m < NB4; ++m) {
                            int o = 0;
#pragma unroll
                            for (int l = 3; l <= p; ++l)
                                if ((m >> (l - 3)) & 1) o += c[l];
                            sum += P[(m * 7 + j) * w + x + (d < 0 ? -o : o)];
                        }
                    }
                    H[r * w + x] = sum;
                }
            }
        } else {
            for (int x = cx; x < w; x += 64) {
#pragma unroll
                for (int q = 0; q < kRowsPer; ++q) {
                    const int r = ry + q * kRowLanes;
                    if (r >= D) break;
                    const int d = r - (n - 1);
                    const int sg = d < 0 ? -1 : 1;
                    const int s = d < 0 ? -d : d;
                    // c[l] = ceil(s_l / 2), s_l = s >> (p - l): what level l adds
                    // to the offset of a row whose bit l-1 is set
                    int c[p + 1];
#pragma unroll
                    for (int l = 1; l <= p; ++l) c[l] = ((s >> (p - l)) + 1) >> 1;
                    int sum = 0;
                    if ((unsigned)(x + d) < (unsigned)w) {
#pragma unroll
                        for (int y = 0; y < N; ++y) {
                            int o = 0;
#pragma unroll
                            for (int l = 1; l <= p; ++l)
                                if ((y >> (l - 1)) & 1) o += c[l];
                            sum += (int)pix[y * w + x + sg * o];
                        }
                    }
                    H[r * w + x] = sum;
                }
            }
        }
        __syncthreads();
        // V_i from V_{i+1} (eqs. (3)-(4)); V_{k-1} is the masked table
        for (int x = cx; x < w; x += 64) {
#pragma unroll
            for (int q = 0; q < kRowsPer; ++q) {
                const int r = ry + q * kRowLanes;
                if (r >= D) break;
                const int c = r * w + x;
                const int xp = x + r - (n - 1);
                const bool valid = (unsigned)xp < (unsigned)w;
                int val = -1;
                if (i == k - 1) {
                    val = valid ? H[c] : -1;
                } else if (valid) {
                    // ascending rows, four reads in flight; a later row wins only
                    // when larger (-2: below every value, -1 marks a missing cell)
                    const int lo = wl[q], hi = wh[q];
                    int m = -2, ia = lo;
                    for (int r0 = lo; r0 <= hi; r0 += 4) {
                        int v[4];
#pragma unroll
                        for (int u = 0; u < 4; ++u)
                            v[u] = r0 + u <= hi ? Vp[(r0 + u) * w + xp] : -2;
#pragma unroll
                        for (int u = 0; u < 4; ++u) {
                            const bool take = v[u] > m;
                            m = take ? v[u] : m;
                            ia = take ? r0 + u : ia;
                        }
                    }
                    val = m >= 0 ? H[c] + m : -1;
                    A[(size_t)i * cells + (size_t)r * w + xp] = (unsigned char)ia;
                }
                if (i == 0) {
                    if (valid) {
                        const unsigned long long kk = small_key(val, x, r, D);
                        best = kk > best ? kk : best;
                    }
                } else {
                    Vc[c] = val;
                }
            }
        }
        __syncthreads();
        int* tmp = Vp;
        Vp = Vc;
        Vc = tmp;
    }
    // the best key of the workgroup: wave maxima, then one thread
    for (int o = 32; o >= 1; o >>= 1) {
        const unsigned long long v = __shfl_xor(best, o, 64);
        best = v > best ? v : best;
    }
    if ((t & 63) == 0) part[t >> 6] = best;
    __syncthreads();
    if (t != 0) return;
    unsigned long long kv = part[0];
    for (int q = 1; q < kSmallThreads / 64; ++q) kv = part[q] > kv ? part[q] : kv;
    const unsigned int lin = 0xffffffffu - (unsigned int)(kv & 0xffffffffull);
    if ((kv >> 32) == 0 || lin / (unsigned int)D >= (unsigned int)w) {
        *a.score = -1;
        return;
    }
    int x = (int)(lin / (unsigned int)D), r = (int)(lin % (unsigned int)D);
    a.xs[0] = x;
    for (int i = 0; i + 1 < k; ++i) {
        x += r - (n - 1);  // x_{i+1}
        a.xs[i + 1] = x;
        r = A[(size_t)i * cells + (size_t)r * w + x];
    }
    a.xs[k] = x + r - (n - 1);
    *a.score = (int)(kv >> 32) - 1;
}

constexpr int kMaxDevices = 64;

// The kernel's dynamic LDS limit, raised once per device (the attribute is
// a property of the function on the current device).
template <typename PixT, int N, int CAP>
hipError_t allow_lds() {
    static std::once_flag once[kMaxDevices];
    static hipError_t rc[kMaxDevices];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
        (void)hipGetLastError();
        return hipErrorInvalidDevice;
    }
    std::call_once(once[dev], [&] {
        rc[dev] = hipFuncSetAttribute(reinterpret_cast<const void*>(&detect_small<PixT, N, CAP>),
                                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)kSmallLds);
    });
    return rc[dev];
}

template <typename PixT, int N, int CAP>
hipError_t launch_small_n(const SmallPack<CAP>& pk, size_t lds, hipStream_t s) {
    hipError_t e = allow_lds<PixT, N, CAP>();
    if (e != hipSuccess) return e;
    TimedLaunch tl("detect_small", s);
    hipLaunchKernelGGL((detect_small<PixT, N, CAP>), dim3(pk.count), dim3(kSmallThreads), lds, s,
                       pk);
    return hipGetLastError();
}

template <typename PixT, int CAP>
hipError_t launch_small_t(int n, const SmallPack<CAP>& pk, size_t lds, hipStream_t s) {
    switch (n) {
        case 1: return launch_small_n<PixT, 1, CAP>(pk, lds, s);
        case 2: return launch_small_n<PixT, 2, CAP>(pk, lds, s);
        case 4: return launch_small_n<PixT, 4, CAP>(pk, lds, s);
        case 8: return launch_small_n<PixT, 8, CAP>(pk, lds, s);
        case 16: return launch_small_n<PixT, 16, CAP>(pk, lds, s);
        case 32: return launch_small_n<PixT, 32, CAP>(pk, lds, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

bool small_apply(const Geometry& g, int dtype, const DpPlan& pl, Pin pin, bool alone) {
    if (!pl.small || pin.j >= 0 || g.n > kSmallMaxN ||
        small_lds_bytes(g.n, g.w, g.k, dtype == 0 ? 1 : 2) > kSmallLds)
        return false;
    // One image alone runs on one CU, bound by its LDS reads (about n + 8 per
    // cell and band; 1.7 + 1.1 us per band at 64 x 64, k = 4), while the
    // general path costs a few launches whatever the size: take the
    // one-workgroup path while its work stays below about 1.25 times that of
    // the 64 x 64 image (4 bands x 31 x 64 cells x 24).  In a batch the
    // images run side by side on separate CUs.
    const long long work = (long long)g.k * g.D * g.w * (g.n + 8);
    return !alone || work <= 240000;
}

hipError_t launch_small_jobs(const SmallJobSpec* jobs, int count, hipStream_t s) {
    // packs of one pixel type and band height
    for (int dtype = 0; dtype < 2; ++dtype)
    for (int n = 1; n <= kSmallMaxN; n *= 2) {
        std::vector<const SmallJobSpec*> group;
        for (int q = 0; q < count; ++q)
            if (jobs[q].dtype == dtype && jobs[q].g.n == n) group.push_back(&jobs[q]);
        for (size_t q0 = 0; q0 < group.size(); q0 += kSmallPack) {
            const int cnt = (int)std::min<size_t>(kSmallPack, group.size() - q0);
            size_t lds = 0;
            auto fill = [&](SmallJob& j, const SmallJobSpec& J) {
                j.img = J.img;
                j.score = J.score;
                j.xs = J.xs;
                j.h = J.g.h;
                j.w = J.g.w;
                j.k = J.g.k;
                j.n = J.g.n;
                j.kind = (int)J.plan.kind;
                j.bound = J.plan.bound;
                j.tan_g = J.plan.tan_gamma;
                lds = std::max(lds, small_lds_bytes(J.g.n, J.g.w, J.g.k, dtype == 0 ? 1 : 2));
            };
            hipError_t e;
            if (cnt == 1) {
                SmallPack<1> pk{};
                fill(pk.job[0], *group[q0]);
                pk.count = 1;
                e = dtype == 0 ? launch_small_t<uint8_t, 1>(n, pk, lds, s)
                               : launch_small_t<uint16_t, 1>(n, pk, lds, s);
            } else {
                SmallPack<kSmallPack> pk{};
                for (int q = 0; q < cnt; ++q) fill(pk.job[q], *group[q0 + q]);
                pk.count = cnt;
                e = dtype == 0 ? launch_small_t<uint8_t, kSmallPack>(n, pk, lds, s)
                               : launch_small_t<uint16_t, kSmallPack>(n, pk, lds, s);
            }
            if (e != hipSuccess) return e;
        }
    }
    return hipSuccess;
}

}  // namespace fhtp
