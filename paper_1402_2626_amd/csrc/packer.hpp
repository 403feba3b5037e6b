// Host-side loading of a system in sparse distributed form: validation,
// canonical order, chunking and the owner-computes slot layout.  Plain C++17
// (no HIP) so it can be built and tested on a machine without a GPU.
#pragma once
#include <cstdint>
#include <string>
#include <vector>

#include "layout.hpp"

namespace pe {

struct SysInput {
  int level = 0;  // level code: limbs 1, 2, 4, plus kRealLevel for real numbers
  int n_vars = 0;
  int n_polys = 0;
  const int64_t* poly_ptr = nullptr;
  const int64_t* mon_ptr = nullptr;
  const int32_t* var_idx = nullptr;
  const int32_t* exps = nullptr;
  const double* coef = nullptr;  // [2][L][M], real: [L][M]
};

// launch shape the packing is made for
struct PackParams {
  int threads = 256;        // workgroup size T
  int seg = 4;              // largest number of variables per lane
  int max_slots = 2048;     // LDS contribution slots per chunk, dummy included
};

struct Packed {
  int level = 0, n = 0, N = 0;  // level: limbs per real part
  int code = 0;                 // level code (limbs, plus kRealLevel for real numbers)
  int64_t M = 0, nnz = 0;
  int emax = 1, kmax = 0;
  PackParams params;
  int max_slots_used = 0;  // largest nslots + 1 (the dummy slot)
  int max_seg_used = 1;
  std::vector<OccRec> occ;
  std::vector<double> mcoef;      // [M][width], packed monomial order (re limbs, then im limbs)
  std::vector<uint32_t> mmeta;    // [M], mon_meta
  std::vector<uint32_t> mon_orig;  // [M]: input index of each packed monomial
  std::vector<uint32_t> occ_orig;  // like occ: input index of each record's
                                   // occurrence (kNoOcc for neutral records)
  std::vector<ChunkDesc> chunks;
  std::vector<uint32_t> chunk_ptr;  // [N+1]
  std::vector<ChunkDesc> rowdesc;   // [N][kRowDesc]: row p's first chunks, zero (count 0) past its last
  std::vector<uint16_t> colptr;     // [chunks][n+1]
  std::vector<int64_t> poly_cost;   // [N] relative cost of a polynomial (for scheduling)
};

// status codes as in the C ABI
constexpr int kOk = 0, kEinval = -1, kEnomem = -2, kEunsupported = -3;

// Checks the input; returns kOk or an error with a message.
int validate(const SysInput& in, std::string& msg);

// Validates and packs.  Returns kOk or an error with a message.
int pack_system(const SysInput& in, const PackParams& pp, Packed& out, std::string& msg);

// lanes per monomial for a monomial of k variables with segments of `seg`
int lanes_for(int k, int seg);

}  // namespace pe
