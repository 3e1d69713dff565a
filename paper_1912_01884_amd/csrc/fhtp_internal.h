// Internal declarations shared by the host API and the kernel translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace fhtp {

// Problem geometry derived from (h, w, k) after validation.
struct Geometry {
    int h, w, k;
    int n;   // band height h/k, a power of two
    int p;   // log2(n)
    int W;   // table width w + n (zero extension of Section 2.1)
    int D;   // shifts per band 2n - 1
    int pitch;  // row pitch (elements) of the DP planes: w rounded up to 64
};

// Brackets a run of `launches` consecutive kernel launches of one family on
// one stream with two events while benchmark timing is on (fhtp_timing_start);
// a no-op otherwise, or when family is null.  Construct it right before the
// first launch; the bracket closes at close() or when it goes out of scope,
// which must come right after the last launch.  One bracket per run rather
// than per launch: every event is a packet of its own between two kernels.
class TimedLaunch {
public:
    TimedLaunch(const char* family, hipStream_t s, int launches = 1);
    ~TimedLaunch() { close(); }
    void close();
    TimedLaunch(const TimedLaunch&) = delete;
    TimedLaunch& operator=(const TimedLaunch&) = delete;

private:
    const char* family_;
    hipStream_t stream_;
    int launches_;
    hipEvent_t begin_ = nullptr;
};

// Largest band height the register FHT kernel handles in one pass.
constexpr int kRegMaxP = 7;

// ---- band tables ------------------------------------------------------------
// Where the band tables of one image live.  Wide: every band [k][D][W] int32
// at `wide`.  Narrow (8-bit pixels and n <= 256, so every line sum is at most
// 256 * 255 < 2^16): bands 0 .. narrow-1 as [narrow][D][W] uint16 at `tab16`,
// the remaining bands (the last one, which the DP reads as V_{k-1}) as int32
// at `wide`.  Narrow tables halve the table traffic of the FHT and the DP.
struct TableSet {
    int32_t* wide = nullptr;
    uint16_t* tab16 = nullptr;
    int narrow = 0;  // bands stored as uint16
};

// Whether a detection of this geometry and pixel type keeps narrow tables.
inline bool narrow_tables_apply(const Geometry& g, int dtype) {
    return dtype == 0 && g.n <= 256 && g.k >= 2;
}

// ---- band FHT -------------------------------------------------------------
// Scratch needed by launch_fht (bytes, 0 when n <= 2^kRegMaxP); dtype 0 =
// uint8 pixels (16-bit scratch cells), 1 = uint16 pixels (32-bit cells).
size_t fht_scratch_bytes(const Geometry& g, int dtype);

// One image's band FHT.
struct FhtJobSpec {
    const void* img;
    int dtype;  // 0 = uint8, 1 = uint16
    Geometry g;
    TableSet tables;
    void* scratch;  // fht_scratch_bytes(g, dtype)
    int grid_mode = 0;  // 0: resident grid looping over the items; 1: one workgroup per item
};
// Band tables of several images, launched in packs that share kernels.
hipError_t launch_fht_jobs(const FhtJobSpec* jobs, int count, hipStream_t stream);
// Writes the tables of one image.  dtype 0 = uint8, 1 = uint16.
hipError_t launch_fht(const void* img, int dtype, const Geometry& g, const TableSet& tables,
                      void* scratch, hipStream_t stream, int grid_mode = 0);

// ---- DP ---------------------------------------------------------------------
// How the DP step takes its range maximum.
enum class WindowKind { Fixed, Generic, Full, Angle };

struct DpPlan {
    WindowKind kind;
    int bound;          // mode 0 shift bound
    double tan_gamma;   // mode 1
    bool a16;           // back-pointers stored as uint16 (D > 256) instead of uint8
    int dc;             // displacements per thread in the fixed-window step (8 or 16)
    int steps = 2;      // most DP steps per launch (1..3) where the window allows them
    int stripe = 16;    // column tiles per stripe of the multi-step kernels' item order
    int fht_grid = 0;   // the detection's FHT: 0 resident grid, 1 one workgroup per item
    bool small = true;  // small images may take the one-workgroup path
};

struct DpBuffers {
    int32_t* vplanes;         // two value planes [2][D][pitch], used in turn
    void* a;                  // back-pointer planes [k-2][D][pitch]
    unsigned long long* key;  // packed argmax keys, one per workgroup of the last step
    int32_t* succ;            // per key: the row d'+n-1 of that cell's best successor
    int32_t* win;             // angle windows lo[D], hi[D]
};

// Through-point restriction: vertex x_j equals x (j = -1: none).
struct Pin {
    int j = -1;
    int x = 0;
};

size_t dp_plane_bytes(const Geometry& g);
size_t dp_backptr_bytes(const Geometry& g, bool a16);
size_t dp_key_count(const Geometry& g);
hipError_t launch_dp(const TableSet& tables, const Geometry& g, const DpPlan& plan,
                     const DpBuffers& buf, int32_t* score, int32_t* xs, hipStream_t stream,
                     Pin pin = Pin{});

// One image's DP, argmax and walk.
struct DpJobSpec {
    TableSet tables;
    Geometry g;
    DpPlan plan;
    DpBuffers buf;
    int32_t* score;
    int32_t* xs;
    Pin pin;
};
// Several images; images of one window class share every step launch.
hipError_t launch_dp_jobs(const DpJobSpec* jobs, int count, hipStream_t stream);

// ---- small images: the whole detection in one workgroup ----------------------
struct SmallJobSpec {
    const void* img;
    int dtype;  // 0 = uint8, 1 = uint16
    Geometry g;
    DpPlan plan;
    int32_t* score;
    int32_t* xs;
};
// Whether a detection runs as one workgroup with everything in LDS (bands of
// at most 32 rows, the image, tables, value planes and back-pointers within
// 64 KB, no pin; alone, i.e. not in a batch, also little enough work).
bool small_apply(const Geometry& g, int dtype, const DpPlan& pl, Pin pin, bool alone);
// Those detections, one workgroup per image, in packs.
hipError_t launch_small_jobs(const SmallJobSpec* jobs, int count, hipStream_t stream);

// ---- optional input steps ---------------------------------------------------
// Detection image from the input: transposed when `transpose` (mostly
// horizontal curves), then each of its rows smoothed with the binomial kernel
// of radius `radius` (0: copy).  Input [h][w]; output [w][h] when transposed,
// else [h][w]; same pixel type.
hipError_t launch_prep(const void* img, int dtype, int h, int w, int radius, int transpose,
                       void* out, hipStream_t stream);

}  // namespace fhtp
