// Internal declarations shared by the HIP translation units of the library.
// Device memory layout (all arrays live in HBM for the whole run):
//   J4     per instance b: Npad[b] x Npad[b] row-major FP64 holding 4*J_ij
//          (zero in the padding); 4*J is exact, it is the pair term of the
//          energy change.
//   h      per instance: Npad[b] FP64.
//   pool   per search s: 2M slots; slot q holds bits[Wmax], E, zob, F[Npmax].
//          A new kept state always takes a slot that the current kept set
//          does not use, so parents stay readable while children are written.
//   kept   per search: up to M slot ids sorted by (E, psi).
//   front  per instance: list of (search, slot) of states to expand.
//   A      per frontier entry: a_i = -2 s_i F_i (the single-flip change).
//   surv   per search: candidate records {E_child, parent slot, i | j<<16}.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace qi {

constexpr int TILE = 64;            // rows of one J tile (one row per lane)
constexpr int TCOL = 32;            // columns of one J tile held in registers
constexpr int MAX_N = 4096;         // pair indices are packed into 16 bits
constexpr int PILOT_K = 48;         // lightest sites used for the per-search pilot cut
constexpr int MERGE_CH = 2048;      // candidates sorted per merge pass (LDS)
constexpr int STAGE = 256;          // wave-private survivor staging (records)
constexpr uint32_t SINGLE = 0xFFFFu;   // j field of a single-flip record
constexpr uint32_t REF_SURV = 0x80000000u;

struct Surv {
    double E;        // energy of the child
    uint32_t code;   // pool slot of the parent: search * 2M + slot
    uint32_t pair;   // i | j << 16, j = SINGLE for a single flip
};
static_assert(sizeof(Surv) == 16, "record layout");

// What the scan needs of one frontier state besides its a_i values.
struct FrRec {
    double T;        // cut - E: a pair survives iff a_i + a_j + 4 s_i s_j J_ij <= T
    double E;        // energy of the state
    int s;           // search
    int code;        // s * 2M + slot
};
static_assert(sizeof(FrRec) == 24, "record layout");

// Everything the kernels need, passed by value.
struct Layout {
    int B, L, M, S;          // instances, searches per instance, kept per search, searches
    int Wmax, Npmax;         // words and padded spins of the largest instance
    int fmax;                // frontier entries per instance (= L*M)
    int cap_surv;            // survivor records per search
    const int* scb;          // [B] frontier states per scan item, per instance (tuned per N)
    const int* N;            // [B]
    const int* Npad;         // [B]
    const long long* joff;   // [B] offset of instance b in J4 (doubles)
    const double* J4;
    const double* h;         // [B][Npmax]
    const uint64_t* zkey;    // [MAX_N] Zobrist keys per site
    // pool
    uint64_t* bits;          // [S][2M][Wmax]
    double* E;               // [S][2M]
    uint64_t* zob;           // [S][2M]
    double* F;               // [S][2M][Npmax]
    uint8_t* fresh;          // [S][2M]
    int* kept;               // [S][M]
    int* nkept;              // [S]
    int* active;             // [S]
    int* retry;              // [S]
    double* cut;             // [S] child energies above this cannot enter
    // frontier
    int* fr_count;           // [B]
    int* fr_list;            // [B][fmax] : s * 2M + slot
    double* A;               // [B][fmax][Npmax]
    FrRec* rec;              // [B][fmax]
    uint64_t* fbits;         // [B][fmax][Wmax] : copy of the state's words
    // survivors
    int* surv_count;         // [S]
    Surv* surv;              // [S][cap_surv]
    // scheduling and counters
    long long* item_prefix;  // [B+1]
    unsigned long long* ctr; // [16] device counters (see CTR_*)
    int* flags;              // [8] per-step flags (see FLAG_*)
    // new kept states of the last merge, for the field update
    int* nm_count;           // [S]
    int* nm_code;            // [S][M] parent slot code
    uint32_t* nm_pair;       // [S][M] i | j << 16
    int* nm_slot;            // [S][M] slot taken by the new state
    // split-bf16 form
    int form;                // 0 plain, 1 split-bf16
    const float* J32;        // per instance, fl32(4J) (same layout as J4)
    const uint16_t* Jhi;     // per instance, bf16(4J)
    const uint16_t* Jlo;     // per instance, bf16(4J - hi)
    const double* ybound;    // [B] max |4J_ij|
    const double* ebf;       // [B] bound on |F~ - F| of the bf16 hi+lo fields
    float* Ft;               // [S][Npmax] F~ of the initial states (bf16 hi+lo GEMM, FP32 sums)
    float* A32;              // [B][fmax][Npmax] fl32(a_i)
    float* RR32;             // [B][fmax][Npmax] T - a_i + slack, rounded up to FP32
    // final merge output
    uint64_t* out_bits;      // [B][M][Wmax]
    double* out_E;           // [B][M]
    int* out_count;          // [B]
};

enum { CTR_PAIRS = 0, CTR_SINGLES = 1, CTR_FRONTIER = 2, CTR_SURV = 3, CTR_RETRY = 4, CTR_STEPS = 5,
       CTR_FALLBACK = 6 };
enum { FLAG_ACTIVE = 0, FLAG_OVERFLOW = 1, FLAG_STUCK = 2, FLAG_RETRY_MODE = 3, FLAG_FIRST = 4 };

__host__ __device__ inline int words_of(int N) { return (N + 63) >> 6; }
__host__ __device__ inline int pad_of(int N) { return (N + TILE - 1) / TILE * TILE; }
// Tiles of 64 rows x 32 columns that hold pairs i < j: row block bi meets
// column blocks bc >= 2*bi of the nc = Npad/32 column blocks.
__host__ __device__ inline long long tiles_of(int N) {
    const long long nb = (N + TILE - 1) / TILE, nc = 2 * nb;
    return nb * nc - nb * (nb - 1);
}

// Host launchers (defined next to their kernels).
hipError_t launch_init_fields(const Layout& lay, const uint64_t* d_x0, hipStream_t st);
hipError_t launch_fields_for(const Layout& lay, int search, int count, hipStream_t st);
hipError_t launch_frontier_plan(const Layout& lay, hipStream_t st);
hipError_t launch_plan_only(const Layout& lay, hipStream_t st);      // re-plan without counting
hipError_t launch_clear_survivors(const Layout& lay, hipStream_t st);
hipError_t launch_prep(const Layout& lay, hipStream_t st);
hipError_t launch_scan(const Layout& lay, int scan_grid, hipStream_t st);
hipError_t launch_merge(const Layout& lay, hipStream_t st);
hipError_t launch_fupdate(const Layout& lay, hipStream_t st);
hipError_t launch_init_split(const Layout& lay, const uint64_t* d_x0, double* d_maxerr, hipStream_t st);
hipError_t launch_prep32(const Layout& lay, hipStream_t st);
hipError_t launch_scan32(const Layout& lay, int scan_grid, hipStream_t st);
hipError_t launch_step_begin(const Layout& lay, bool retry_mode, hipStream_t st);
hipError_t launch_final(const Layout& lay, hipStream_t st);

}  // namespace qi
