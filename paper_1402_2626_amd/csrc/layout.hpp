// Device-side layout of a packed system.  Shared by the host packer and the
// kernels; plain C++ so the packer builds without HIP.
//
// A polynomial's monomials are cut into CHUNKS.  A chunk is processed by one
// workgroup in one pass: every monomial of the chunk gets a group of `s`
// consecutive lanes (s a power of two, at most one wavefront), lane q of the
// group handles a contiguous segment of at most `seg` of the monomial's
// variables, and each partial derivative (and the monomial's value) is written
// to its own LDS SLOT.  Slots are numbered so that the contributions to one
// output column are contiguous: column c owns slots colptr[c] ..
// colptr[c+1]-1.  Columns 0..n-1 are the Jacobian columns; columns
// fcol..fcol+R-1 (fcol >= n, the block inside one aligned run of 64 columns)
// are R partial sums of F (monomial g of a chunk adds its value to column
// fcol + g % R), summed in order at the end; columns between n and fcol stay
// empty.  This owner-computes order is fixed at load time, so results are
// bitwise reproducible.
#pragma once
#include <cstdint>

namespace pe {

// one occurrence of a variable in a monomial, stored lane-major per chunk:
// record i of lane lam of chunk ch is at occ[ch.occ_base + i * ch.width + lam]
struct OccRec {
  uint16_t var;   // variable index
  uint16_t exp;   // exponent (>= 1)
  uint16_t slot;  // LDS slot of this partial derivative within the chunk
  uint16_t pad;
};

struct ChunkDesc {
  uint32_t occ_base;     // first OccRec of the chunk
  uint32_t mon_base;     // first monomial (packed order) of the chunk
  uint32_t colptr_base;  // first colptr entry of the chunk (ncols + 1 entries)
  uint32_t poly;         // polynomial the chunk belongs to
  uint16_t count;        // monomials in the chunk
  uint16_t nslots;       // slots used
  uint16_t width;        // lanes used = count * s (the OccRec row stride)
  uint8_t s;             // lanes per monomial (power of two, <= 64)
  uint8_t seg;           // records per lane = ceil(kmax / s)
};

// per-monomial metadata (packed order): k in the low 16 bits, F slot high
inline uint32_t mon_meta(uint32_t k, uint32_t fslot) { return k | (fslot << 16); }

constexpr int kMaxVars = 65535;
constexpr int kMaxSeg = 16;      // largest segment any kernel variant handles
constexpr int kMaxWave = 64;     // lanes per wavefront on gfx950
constexpr int kMaxMonomialVars = kMaxWave * kMaxSeg;  // 1024

}  // namespace pe
