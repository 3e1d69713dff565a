// Optional input steps before the band FHT: the transpose that turns mostly
// horizontal curves into mostly vertical ones (Fig. 7), and the row-wise
// smoothing of the main problem's step 1.
//
// Smoothing reads the Gaussian of step 1 as the binomial kernel C(2r, i),
// i = 0 .. 2r (variance r/2), with each row extended by repeating its end
// pixels and the sum normalised by 4^r with rounding half up, so the whole
// path stays exact integer arithmetic and the result keeps the pixel type.
//
// One workgroup makes a 64 x 64 tile of the detection image.  It stages the
// source rows of the tile plus an r-column halo in LDS, reading the input
// along its own rows (so the transposed case reads coalesced too), then each
// thread produces 16 outputs of one column, storing along rows.
#include "fhtp_internal.h"

namespace fhtp {
namespace {

constexpr int kTile = 64;
constexpr int kMaxRadius = 7;
constexpr int kThreads = 256;

struct PrepArgs {
    const void* img;
    void* out;
    int hs, ws;     // input dimensions
    int ho, wo;     // detection image dimensions
    int radius;
    int shift;      // 2 * radius
    int transpose;
    int coef[2 * kMaxRadius + 1];
};

template <typename PixT>
__global__ __launch_bounds__(kThreads) void prep_kernel(PrepArgs a) {
    constexpr int kPitch = kTile + 2 * kMaxRadius + 1;  // odd: no bank conflicts either way
    __shared__ int tile[kTile * kPitch];
    const PixT* __restrict__ img = static_cast<const PixT*>(a.img);
    PixT* __restrict__ out = static_cast<PixT*>(a.out);
    const int r = a.radius;
    const int span = kTile + 2 * r;
    const int x0 = blockIdx.x * kTile;  // detection columns of the tile
    const int lxo = threadIdx.x & (kTile - 1);
    const int half = r > 0 ? 1 << (a.shift - 1) : 0;
    for (int y0 = blockIdx.y * kTile; y0 < a.ho; y0 += gridDim.y * kTile) {
        const int rows = min(kTile, a.ho - y0);
        __syncthreads();  // the previous tile's readers are done
        // Stage S(y, x) for y in [y0, y0 + rows), x in [x0 - r, x0 + 64 + r), x clamped.
        if (!a.transpose) {
            for (int t = threadIdx.x; t < rows * span; t += kThreads) {
                const int ly = t / span, lx = t - ly * span;
                const int x = min(max(x0 - r + lx, 0), a.wo - 1);
                tile[ly * kPitch + lx] = img[(size_t)(y0 + ly) * a.ws + x];
            }
        } else {
            // S(y, x) = input(x, y): consecutive threads take consecutive y,
            // which are consecutive pixels of one input row.
            for (int t = threadIdx.x; t < rows * span; t += kThreads) {
                const int lx = t / rows, ly = t - lx * rows;
                const int x = min(max(x0 - r + lx, 0), a.wo - 1);
                tile[ly * kPitch + lx] = img[(size_t)x * a.ws + (y0 + ly)];
            }
        }
        __syncthreads();
        const int x = x0 + lxo;
        if (x < a.wo) {
            for (int ly = threadIdx.x >> 6; ly < rows; ly += kThreads / kTile) {
                const int* row = tile + ly * kPitch + lxo;
                int acc = 0;
#pragma unroll
                for (int i = 0; i <= 2 * kMaxRadius; ++i)
                    if (i <= 2 * r) acc += a.coef[i] * row[i];
                out[(size_t)(y0 + ly) * a.wo + x] = (PixT)((acc + half) >> a.shift);
            }
        }
    }
}

}  // namespace

hipError_t launch_prep(const void* img, int dtype, int h, int w, int radius, int transpose,
                       void* out, hipStream_t stream) {
    if (radius < 0 || radius > kMaxRadius) return hipErrorInvalidValue;
    PrepArgs a{};
    a.img = img;
    a.out = out;
    a.hs = h;
    a.ws = w;
    a.ho = transpose ? w : h;
    a.wo = transpose ? h : w;
    a.radius = radius;
    a.shift = 2 * radius;
    a.transpose = transpose;
    a.coef[0] = 1;
    for (int i = 1; i <= 2 * radius; ++i) a.coef[i] = a.coef[i - 1] * (2 * radius - i + 1) / i;
    const int tiles_y = (a.ho + kTile - 1) / kTile;
    const dim3 grid((a.wo + kTile - 1) / kTile, tiles_y < 65535 ? tiles_y : 65535);
    TimedLaunch tl("prep_kernel", stream);
    if (dtype == 0)
        hipLaunchKernelGGL(prep_kernel<uint8_t>, grid, dim3(kThreads), 0, stream, a);
    else
        hipLaunchKernelGGL(prep_kernel<uint16_t>, grid, dim3(kThreads), 0, stream, a);
    return hipGetLastError();
}

}  // namespace fhtp
