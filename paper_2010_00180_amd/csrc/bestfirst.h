// The best-first search of Alg. 2-4 (k_bestfirst.hip): its arguments and
// the split of a block's arrays between LDS and global memory.
#pragma once

#include "common.h"

namespace qi {

constexpr int BFS_NMAX = 64;       // one word per state
constexpr int BFS_K1MAX = 1 << 20; // list entries (K + 1) at most (lists past the LDS go to global memory)
constexpr size_t BFS_LDS_MAX = 160 * 1024;

struct BestFirstArgs {
    int L, K1, I, Cs, h1;      // searches per instance, list entries, iterations, offered-entry room of a
                               // search (a power of two, at least its children), H1 mode
    const int* N;              // [B]
    const long long* joff;     // [B] offset of instance b's N*N couplings in J
    const double* J;           // J_ij, row-major per instance
    const double* h;           // [B][64]
    const uint64_t* x0;        // [B*L] initial states
    uint64_t* out_psi;         // [B*L][K1] final lists (placeholders have E = +inf)
    double* out_E;
    uint8_t* out_used;
    int* out_born;
    int* out_expanded;         // [B*L] iterations that expanded a state
    uint64_t* merged_psi;      // [B][K1] Alg. 4 result
    double* merged_E;
    // what does not fit in LDS goes to global memory, ws_stride bytes per
    // block: a search's lists and hash, or all of a merge block's arrays
    int lists_in_lds, merge_in_lds;
    unsigned char* ws;
    size_t ws_stride;
};

// dynamic LDS of the two kernels and the global bytes per block (0: none)
struct BestFirstPlan {
    size_t lds_search, lds_merge, ws_stride;
    int lists_in_lds, merge_in_lds;
};

BestFirstPlan bestfirst_plan(int K1, int Cs);
hipError_t bestfirst_set_lds(const BestFirstPlan& p);
hipError_t launch_bestfirst(const BestFirstArgs& a, int n_inst, const BestFirstPlan& p, hipStream_t st);

}  // namespace qi
