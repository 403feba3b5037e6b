// Device-side layout of a packed system.  Shared by the host packer and the
// kernels; plain C++ so the packer builds without HIP.
//
// A polynomial's monomials are cut into CHUNKS.  A chunk is processed by one
// workgroup in one pass: every monomial of the chunk gets a group of `s`
// consecutive lanes (s a power of two, at most one wavefront), lane q of the
// group handles the SEGMENT of the monomial's occurrences q, q + s, q + 2s, ...
// (at most `seg` of them; occurrences in variable order), and each partial
// derivative is written to its own LDS SLOT.
// Slots are numbered so that the contributions to one Jacobian column are
// contiguous: column c owns slots colptr[c] .. colptr[c+1]-1.  This
// owner-computes order is fixed at load time, so results are bitwise
// reproducible.  Every lane walks all `seg` records of the chunk: positions
// past the end of its segment hold a neutral record (variable n, which the
// kernels read as the constant 1, exponent 1, and the chunk's dummy slot
// `nslots`, which no column owns).  The monomial values (the terms of F) do
// not go through slots.
#pragma once
#include <cstdint>

namespace pe {

// one occurrence of a variable in a monomial, stored lane-major per chunk:
// record i of lane lam of chunk ch is at occ[ch.occ_base + i * ch.width + lam]
struct alignas(8) OccRec {
  uint16_t var;   // variable index
  uint16_t exp;   // exponent (>= 1)
  uint16_t slot;  // LDS slot of this partial derivative within the chunk (nslots: dummy)
  uint16_t pad;
};

struct ChunkDesc {
  uint32_t occ_base;     // first OccRec of the chunk
  uint32_t mon_base;     // first monomial (packed order) of the chunk
  uint32_t colptr_base;  // first colptr entry of the chunk (n + 1 entries)
  uint32_t poly;         // polynomial the chunk belongs to
  uint16_t count;        // monomials in the chunk
  uint16_t nslots;       // slots used; slot nslots is the dummy
  uint16_t width;        // lanes used = count * s (the OccRec row stride)
  uint8_t s;             // lanes per monomial (power of two, <= 64)
  uint8_t seg;           // records per lane = ceil(kmax / s)
};

// per-monomial metadata (packed order): the number of variables k
inline uint32_t mon_meta(uint32_t k) { return k; }

constexpr int kRealLevel = 8;  // flag of the level code for real numbers
constexpr uint32_t kNoOcc = 0xffffffffu;  // input occurrence index of a neutral record
constexpr int kRowDesc = 4;      // first chunk descriptors of each row, stored by row
constexpr int kMaxVars = 65535;
constexpr int kMaxSeg = 16;      // largest segment any kernel variant handles
constexpr int kMaxWave = 64;     // lanes per wavefront on gfx950
constexpr int kMaxMonomialVars = kMaxWave * kMaxSeg;  // 1024

}  // namespace pe
