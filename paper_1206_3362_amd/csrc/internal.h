// Internal declarations shared by the host and device translation units of
// libfwbf.so.  Not part of the public ABI (include/fwbf.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/fwbf.h"

namespace fwbf {

// Thread-local error message; returns `code` for convenience.
int fail(int code, const std::string &msg);
int hip_fail(hipError_t e, const char *what);

// Compact adjacency of the QC base, used by the kernels.
//   col entry (block column j, t-th circulant permutation): (i << 24) | (q << 16) | s
//     where q is the position of the same permutation in row i's list.
//   row entry (block row i, q-th circulant permutation):   (j << 16) | s
// A block with several shifts contributes one entry per shift, listed in
// descending shift order; blocks come in ascending block row / column order.
struct DeviceTables {
    uint32_t *col = nullptr;  // nb * dv_max
    uint32_t *row = nullptr;  // mb * dc_max
    uint8_t *coldeg = nullptr;  // nb
    uint8_t *rowdeg = nullptr;  // mb
    uint32_t *shift = nullptr;  // mb * nb raw shifts (-1 as 0xFFFFFFFF)
};

}  // namespace fwbf

struct fwbf_code {
    int Z = 0, mb = 0, nb = 0, N = 0, M = 0;
    int dv_max = 0, dc_max = 0;
    std::vector<int> shift;  // mb * nb: the block's largest shift, -1 = zero block
    std::vector<std::vector<int>> cells;  // mb * nb shift lists, descending
    bool multi = false;  // some block holds more than one shift
    std::vector<uint32_t> col, row;
    std::vector<uint8_t> coldeg, rowdeg;

    // GF(2) reduced row-echelon form (lazy)
    std::once_flag rref_once;
    int rref_rc = 0;
    int rank = 0, K = 0, words = 0;
    std::vector<uint64_t> rref;  // rank rows x words
    std::vector<int> piv, info;

    // device copies of the compact tables, one per device
    std::mutex mu;
    std::map<int, fwbf::DeviceTables> dev;
};

namespace fwbf {
// Returns the device tables of `code` on the current device (uploaded on
// first use; synchronous upload, done once per code and device).
int device_tables(fwbf_code *code, DeviceTables *out);
// The same tables only if already uploaded to the current device (never
// allocates); FWBF_E_INVALID otherwise.
int device_tables_resident(const fwbf_code *code, DeviceTables *out);
int ensure_rref(fwbf_code *code);
}  // namespace fwbf
