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
//   surv   per search: candidate records {E_child, frontier entry, i | j<<16}.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace qi {

constexpr int TILE = 64;            // rows/cols of one J tile (one row per lane)
constexpr int MAX_N = 4096;         // pair indices are packed into 16 bits
constexpr int PILOT_K = 48;         // lightest sites used for the per-search pilot cut
constexpr int MERGE_CH = 4096;      // candidates sorted per merge pass (LDS)
constexpr int STAGE = 512;          // wave-private survivor staging (records)
constexpr uint32_t SINGLE = 0xFFFFu;   // j field of a single-flip record
constexpr uint32_t REF_SURV = 0x80000000u;

struct Surv {
    double E;        // energy of the child
    uint32_t f;      // frontier entry (index within its instance's list)
    uint32_t pair;   // i | j << 16, j = SINGLE for a single flip
};
static_assert(sizeof(Surv) == 16, "record layout");

// Everything the kernels need, passed by value.
struct Layout {
    int B, L, M, S;          // instances, searches per instance, kept per search, searches
    int Wmax, Npmax;         // words and padded spins of the largest instance
    int fmax;                // frontier entries per instance (= L*M)
    int cap_surv;            // survivor records per search
    int sc;                  // frontier states per scan item
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
    double* T;               // [B][fmax] : cut[s] - E (scan threshold on a_i + a_j + sJ)
    // survivors
    int* surv_count;         // [S]
    Surv* surv;              // [S][cap_surv]
    // scheduling and counters
    long long* item_prefix;  // [B+1]
    unsigned long long* ctr; // [16] device counters (see CTR_*)
    int* flags;              // [8] per-step flags (see FLAG_*)
    // final merge output
    uint64_t* out_bits;      // [B][M][Wmax]
    double* out_E;           // [B][M]
    int* out_count;          // [B]
};

enum { CTR_PAIRS = 0, CTR_SINGLES = 1, CTR_FRONTIER = 2, CTR_SURV = 3, CTR_RETRY = 4, CTR_STEPS = 5,
       CTR_FALLBACK = 6 };
enum { FLAG_ACTIVE = 0, FLAG_OVERFLOW = 1, FLAG_STUCK = 2, FLAG_RETRY_MODE = 3 };

__host__ __device__ inline int words_of(int N) { return (N + 63) >> 6; }
__host__ __device__ inline int pad_of(int N) { return (N + TILE - 1) / TILE * TILE; }
__host__ __device__ inline long long tiles_of(int N) {
    long long nb = (N + TILE - 1) / TILE;
    return nb * (nb + 1) / 2;
}

// Host launchers (defined next to their kernels).
hipError_t launch_init_fields(const Layout& lay, const uint64_t* d_x0, hipStream_t st);
hipError_t launch_fields_for(const Layout& lay, int search, int count, hipStream_t st);
hipError_t launch_step(const Layout& lay, int scan_grid, bool retry_mode, hipStream_t st);
hipError_t launch_step_begin(const Layout& lay, bool retry_mode, hipStream_t st);
hipError_t launch_final(const Layout& lay, hipStream_t st);

}  // namespace qi
