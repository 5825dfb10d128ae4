// Internal declarations of libmips shared by the host-side files: the
// device control block, the launch plans and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/mips.h"

namespace mips {

// Precision codes (same values as the public mips_precision enum).  The
// public code PREC_FP8_CASCADE selects the E4M3 screen whose candidates are
// re-screened in bfloat16 before the float64 rescore; every kernel sees the
// screen precision PREC_FP8 and a separate cascade flag.
enum { PREC_FP32 = 0, PREC_BF16 = 1, PREC_FP8 = 2, PREC_FP8_CASCADE = 3 };

inline int screen_prec(int p) { return p == PREC_FP8_CASCADE ? PREC_FP8 : p; }
inline bool cascade_of(int p) { return p == PREC_FP8_CASCADE; }
inline bool valid_prec(int p) { return p >= PREC_FP32 && p <= PREC_FP8_CASCADE; }

// User blocks of 32 per screen wave.  Each user block holds its operand
// registers, an accumulator tile and a KM-entry K-list.  The bfloat16 brute
// force takes four blocks (128 users: each item tile loaded once per 128
// users) up to 64 factors and 16 list entries (E4M3, with its hundreds of
// candidates per user, was measured slower so); otherwise two blocks up to a
// 32-entry list, except for the float32 screen past 16 entries or 32 chunks
// and the bfloat16 screen with a 32-entry list over 8 chunks.  The walk
// (stops = true) keeps at most two blocks, since a wave runs until its
// slowest user stops and a walk is a few tiles long; the norm-pruned brute
// force takes the brute force's count (four blocks measured 1.66 -> 1.52 ms
// against two on 480,000 x 17,770, BF16, K = 10: each item tile serves 128
// users, and its stop test still ends waves early).
__host__ __device__ constexpr int ub_for(int prec, int km, int nch_cap, bool stops) {
    return (!stops && prec == PREC_BF16 && km <= 16 && nch_cap <= 4)
               ? 4
               : (prec == PREC_FP32
                      ? ((km <= 16 && nch_cap <= 32) ? 2 : 1)
                      : (km <= 16 ? 2 : ((km <= 32 && !(prec == PREC_BF16 && nch_cap >= 8)) ? 2 : 1)));
}

// Certification runs at the end of the screen kernel when the K-list fits a
// small sorted register list, an even number of user blocks keeps every lane
// busy (one user per lane and pass), and the screen keeps few candidates per
// user (not E4M3, whose hundreds of candidates per user make one lane per
// user too slow; there the separate kernel spreads a user over 16 or 64
// lanes).
__host__ __device__ constexpr bool fused_certify(int prec, int km, int ub) {
    return prec != PREC_FP8 && km <= 16 && ub % 2 == 0;
}

// Candidate lists: each lane of a screen wave appends to a list of its own
// (cap entries).  Element-major where the screen kernel certifies its own
// users (FP32/BF16, K <= 16): entry j of lane l of user block blk sits at
// (blk cap + j) 64 + l, so the j-th entries of a block's 64 lanes are
// contiguous and the fused certification, one lane per user, reads 512
// contiguous bytes per entry.  Lane-major where a certification kernel reads
// them (E4M3, K > 16, one user block per wave): at (blk 64 + l) cap + j, so
// a lane's stores fill its own cache lines and the kernel's lanes, reading
// consecutive entries of one list, read contiguous memory.  cand_base gives
// entry 0 of a lane's list; entry j is cand_stride entries further on.
constexpr int kCandStride = 64;
__host__ __device__ inline int64_t cand_base(int64_t blk, int lane, int cap, bool lane_major) {
    return lane_major ? ((blk << 6) + lane) * cap : ((blk * cap) << 6) + lane;
}
__host__ __device__ inline int cand_stride(bool lane_major) { return lane_major ? 1 : kCandStride; }
inline size_t cand_bytes(int64_t n_ublk, int cap) { return (size_t)n_ublk * 64 * cap * 8; }


// Device-resident control block of one call.  Zeroed at the start of every
// call by a fill kernel (never by a memset node, so callers may capture the
// call in a graph).
struct Ctrl {
    unsigned int nonfinite;          // any NaN/Inf seen in U or I
    unsigned int fb_count;           // users appended to the fallback list
    unsigned int cmax_bits;          // max_i ||i|| (rounded up), float bits
    unsigned int emax_bits;          // max_i ||screen(i)||, float bits
    unsigned int gmax_bits;          // max_i G_i, float bits
    unsigned int bad_index;          // backward: idx entries out of range
    unsigned long long cand_total;   // candidates appended by the screen
    unsigned long long cand_max;     // max candidates of one user
    unsigned long long rescored;     // pairs rescored in float64
    unsigned long long visited;      // items scored, summed over users
    unsigned long long max_abs_err;  // float64 bits of max |s - key|
    unsigned long long max_rel_err;  // float64 bits of max |s - key| / (||u|| ||i||)
};

// Shape of the screen for one call.
struct ScreenPlan {
    int prec = 0;
    int f = 0, f_pad = 0, nch = 0;   // factors, padded factors, matrix-core K-chunks
    int K = 0, KM = 0, UB = 0;       // K, register K-list length, user blocks per wave
    int NCH = 0;                     // compiled chunk capacity (>= nch)
    int cap = 0;                     // candidate slots per lane
    int kc = 0;                      // kept-candidate slots per lane in certification
    bool fast = false;               // false: every user goes to the exact fallback kernel
    int64_t n_u = 0, n_i = 0;
    int64_t n_blk = 0, n_i_pad = 0;  // item tiles of 32, padded item count
    int64_t n_waves = 0;             // waves of the screen / certification grid
    int64_t n_ublk = 0;              // n_waves * UB
    int fb_grid = 0;                 // workgroups of the fallback kernel
    float gamma = 0.0f;              // accumulation error factor of the screen
};

// Parameters shared by the screen (score tiles + streaming top-K) kernel and
// the certification kernel.  `walk` selects the Maximus list walk.
struct ScreenArgs {
    const float* U;
    const float* I;
    int64_t n_u, n_i, n_blk, n_i_pad;
    int f, f_pad, nch, K, cap, kc;
    float gamma;
    // brute force: items in norm order, packed in matrix-core operand order
    const void* packed;
    const int* pscale;        // FP8: E8M0 scale byte per sorted position
    const float2* blockmax;   // per item tile: (max C, max G)
    const int* perm;          // sorted position -> item index (-1 past the last item)
    const float4* cgpos;      // (C_i, G_i, item bits, 0) by sorted position
    const float* tailmax;     // per tile: max ||i|| over this and all later tiles
    int prune;                // norm pruning: a user stops once ||u|| tailmax < tau_u
    // Maximus walk
    int walk;
    int warm_rounds;          // warm-up rounds seeding tau (tiles per warm-up set)
    int shared_blocks;        // leading list tiles scored before any user may stop
    const int4* tiles;        // (cluster, first sorted user, user count, 0)
    const int* sorted_users;  // users grouped by cluster
    const int* lists;         // C x n_i item indices in walk order
    const float* lbound;      // C x n_i_pad rounded-up bounds in walk order (+ -inf pad)
    const float2* cblockmax;  // C x n_blk per-tile maxima in walk order
    const void* qrow;         // n_i x f_pad screen copies by item index
    const int* kexp;          // FP8: row scale exponent by item index
    // the first wpre tiles of every cluster's list, packed in matrix-core
    // operand order ([cluster][tile][chunk][lane]) with their per-row (C, G)
    // and, for E4M3, E8M0 scale bytes ([cluster][tile][row]): a walk tile
    // below wpre loads without a gather through the list
    int wpre;
    const void* wpacked;
    const float2* wcg;
    const int* wscale;
    // per-item scalars by item index
    const float* Corig;       // ||i|| rounded up
    const float* Gorig;       // ||i - screen(i)|| + gamma ||screen(i)||, rounded up
    // E4M3 certification cascade: a bfloat16 re-screen of the candidates
    // before the float64 rescore (qrow_b null: no cascade)
    const void* qrow_b;       // n_i x fpb bfloat16 copies by item index
    const float* Gorig_b;     // ||i - bf16(i)|| + gamma_b ||bf16(i)||, rounded up
    const unsigned int* maxb; // float bits of max ||i||, max ||bf16(i)||, max Gorig_b
    int fpb;                  // bfloat16 row stride (multiple of 8, >= f)
    // per-call state
    int want_stats;           // accumulate the optional statistics (atomics)
    Ctrl* ctrl;
    int* uflag;               // n_u: 0 normal, 1 on the fallback list
    int* flist;               // n_u: fallback list
    float4* uscal;            // n_u: (A_u, B_u, slack_u, tau_u)
    int64_t n_ublk;           // user blocks with candidate storage
    int* cnt;                 // n_ublk * 64 candidate counts
    int cand_lm;              // candidate lists lane-major (the E4M3 screen) or element-major
    int2* cand;               // n_ublk * 64 lists of cap candidates (score bits, reference):
                              // the reference is the item (walk) or the sorted position
                              // (brute force), see cand_item
    int32_t* out_idx;
    double* out_score;
};

// Item index named by a candidate entry's reference (-1 stays -1).
__device__ inline int cand_item(const ScreenArgs& a, int ref) {
    return (a.walk || ref < 0) ? ref : a.perm[ref];
}

struct FallbackArgs {
    const float* U;
    const float* I;
    int64_t n_u, n_i;
    int f, K;
    const int* flist;
    Ctrl* ctrl;
    double* keys;             // fb_grid x n_i scratch
    int pre_users;            // fallback users whose keys a separate kernel computed
    int32_t* out_idx;
    double* out_score;
};

// Walk prefix tiles of a Maximus index (see ScreenArgs::wpacked).
struct WalkPackArgs {
    const int* lists;         // C x n_i_pad walk lists (-1 past the last item)
    int64_t n_i_pad;
    int wpre, f_pad, nch;
    const void* qrow;         // screen copies by item index
    const int* kexp;          // E4M3 row scale exponents (null otherwise)
    const float* Corig;
    const float* Gorig;
    void* packed;
    float2* cg;
    int* scale;
};

struct ItemPrepArgs {
    const float* I;
    int64_t n_i, n_blk;
    int f, f_pad, nch;
    float gamma;
    float* Corig;
    float* Gorig;
    float* Eorig;
    int* kexp;
    void* qrow;
    int* bucket;
    unsigned int* hist;       // 4096 bucket counts, then 4096 offsets
    int* perm;
    void* packed;
    int* pscale;
    float2* blockmax;
    float4* cgpos;            // (C_i, G_i, item bits, 0) by sorted position (nullable)
    Ctrl* ctrl;
};

constexpr int kBuckets = 4096;
constexpr int kFallbackMaxK = 4096;

// Launchers (each returns hipSuccess or the launch error).
hipError_t launch_zero(void* p, size_t bytes, hipStream_t s);
hipError_t launch_scan4096(unsigned int* hist, hipStream_t s);
hipError_t launch_tailmax(const float2* blockmax, int64_t n_blk, float* tailmax, hipStream_t s);
hipError_t launch_item_prep(int prec, const ItemPrepArgs& a, bool pack, hipStream_t s);
// norms and screen copies of the same items for up to three precisions in
// one pass (a[p] null: precision p skipped)
hipError_t launch_item_stats3(const ItemPrepArgs* const (&a)[3], hipStream_t s);
// walk prefix tiles of C clusters (grid wpre x C)
hipError_t launch_walk_pack(int prec, const WalkPackArgs& a, int C, hipStream_t s);
hipError_t launch_screen(const ScreenPlan& p, const ScreenArgs& a, hipStream_t s);
hipError_t launch_screen_fp32(const ScreenPlan& p, const ScreenArgs& a, hipStream_t s);
hipError_t launch_screen_bf16(const ScreenPlan& p, const ScreenArgs& a, hipStream_t s);
hipError_t launch_screen_fp8(const ScreenPlan& p, const ScreenArgs& a, hipStream_t s);
hipError_t launch_certify(const ScreenPlan& p, const ScreenArgs& a, hipStream_t s);
hipError_t launch_flag_all(int64_t n_u, int* uflag, int* flist, Ctrl* ctrl, hipStream_t s);
hipError_t launch_fallback(const ScreenPlan& p, const FallbackArgs& a, hipStream_t s);

// scratch: backward_scratch_bytes(n_i, n_u K) bytes of device memory, or null
// for stream-ordered scratch allocated and released on `s`
size_t backward_scratch_bytes(int64_t n_i, int64_t npairs);
hipError_t launch_backward(const float* U, const float* I, int64_t n_u, int64_t n_i, int f, int K,
                           const int32_t* idx, const float* G, float* dU, float* dI,
                           void* scratch, hipStream_t s);
hipError_t launch_nonfinite_scan(const float* U, int64_t nu_elems, const float* I,
                                 int64_t ni_elems, Ctrl* ctrl, hipStream_t s);

// Host-side helpers of the C ABI.
// Device memory of the current device from the library's block cache: the
// block holds at least `bytes` (*bytes_out: its size, to pass back on
// release).  Release a block only when no work on the device can still use
// it.
hipError_t cache_alloc(void** p, size_t* bytes_out, size_t bytes);
void cache_release(void* p, size_t bytes);

int fail(int code, const char* fmt, ...);
int hip_fail(hipError_t e, const char* what);

// Brackets the kernels launched in its scope with HIP events on `s` while
// kernel timing is enabled (mips_profile_enable); otherwise does nothing.
class PhaseTimer {
public:
    PhaseTimer(int phase, hipStream_t s);
    ~PhaseTimer();
    PhaseTimer(const PhaseTimer&) = delete;
    PhaseTimer& operator=(const PhaseTimer&) = delete;
private:
    int phase_;
    hipStream_t stream_;
    hipEvent_t start_ = nullptr, stop_ = nullptr;
    bool active_ = false;
};

// Test knobs set through mips_debug_set (0 = normal operation): a smaller
// number of candidate slots per lane, and the certification kernel to use
// (1 one wave per user, 2 a group of lanes per user).
int debug_cand_cap();
int debug_certify_kernel();

// Copies the control block to the host (synchronising `s`) and fills the
// public statistics struct.
int finish_stats(Ctrl* dctrl, hipStream_t s, int64_t n_u, int64_t n_i, mips_stats* stats);

// Plan selection (host only).
bool make_screen_plan(int64_t n_u, int64_t n_i, int f, int K, int prec, bool stops,
                      ScreenPlan* out);

}  // namespace mips
