// Host build of the library's packer for invariant checks from the test
// suite: packs a system and returns the packed arrays.
#include <cstdint>
#include <cstring>
#include <string>
#include "../paper_1402_2626_amd/csrc/packer.hpp"

using namespace pe;

static Packed g_packed;
static std::string g_msg;

extern "C" int pe_test_pack(int level, int n, int N, const int64_t* poly_ptr, const int64_t* mon_ptr,
                            const int32_t* var_idx, const int32_t* exps, const double* coef, int seg, int max_slots,
                            int64_t* sizes /* [9] */) {
  SysInput in;
  in.level = level;
  in.n_vars = n;
  in.n_polys = N;
  in.poly_ptr = poly_ptr;
  in.mon_ptr = mon_ptr;
  in.var_idx = var_idx;
  in.exps = exps;
  in.coef = coef;
  PackParams pp;
  pp.threads = 256;
  pp.seg = seg;
  pp.max_slots = max_slots;
  int st = pack_system(in, pp, g_packed, g_msg);
  if (st != 0) return st;
  sizes[0] = int64_t(g_packed.chunks.size());
  sizes[1] = int64_t(g_packed.occ.size());
  sizes[2] = int64_t(g_packed.colptr.size());
  sizes[3] = g_packed.M;
  sizes[4] = g_packed.n;
  sizes[5] = g_packed.max_slots_used;
  sizes[6] = g_packed.emax;
  sizes[7] = g_packed.kmax;
  sizes[8] = 0;
  return 0;
}

extern "C" const char* pe_test_pack_msg() { return g_msg.c_str(); }

// row-ordered first descriptors as 9 int64 each, kRowDesc per row
extern "C" int pe_test_pack_rowdesc(int64_t* out) {
  for (size_t i = 0; i < g_packed.rowdesc.size(); ++i) {
    const ChunkDesc& c = g_packed.rowdesc[i];
    int64_t* o = out + 9 * i;
    o[0] = c.occ_base; o[1] = c.mon_base; o[2] = c.colptr_base; o[3] = c.poly; o[4] = c.count;
    o[5] = c.nslots; o[6] = c.width; o[7] = c.s; o[8] = c.seg;
  }
  return kRowDesc;
}

// chunks as 9 int64 each: occ_base, mon_base, colptr_base, poly, count, nslots, width, s, seg
extern "C" void pe_test_pack_get(int64_t* chunks, uint16_t* occ /* [occ][4] */, uint16_t* colptr, uint32_t* mmeta,
                                 double* mcoef, uint32_t* chunk_ptr) {
  for (size_t i = 0; i < g_packed.chunks.size(); ++i) {
    const ChunkDesc& c = g_packed.chunks[i];
    int64_t* o = chunks + 9 * i;
    o[0] = c.occ_base; o[1] = c.mon_base; o[2] = c.colptr_base; o[3] = c.poly; o[4] = c.count;
    o[5] = c.nslots; o[6] = c.width; o[7] = c.s; o[8] = c.seg;
  }
  std::memcpy(occ, g_packed.occ.data(), g_packed.occ.size() * sizeof(OccRec));
  std::memcpy(colptr, g_packed.colptr.data(), g_packed.colptr.size() * 2);
  std::memcpy(mmeta, g_packed.mmeta.data(), g_packed.mmeta.size() * 4);
  std::memcpy(mcoef, g_packed.mcoef.data(), g_packed.mcoef.size() * 8);
  std::memcpy(chunk_ptr, g_packed.chunk_ptr.data(), g_packed.chunk_ptr.size() * 4);
}

// input-order maps: [M] monomial indices, [occ] occurrence indices
extern "C" void pe_test_pack_orig(uint32_t* mon_orig, uint32_t* occ_orig) {
  std::memcpy(mon_orig, g_packed.mon_orig.data(), g_packed.mon_orig.size() * 4);
  std::memcpy(occ_orig, g_packed.occ_orig.data(), g_packed.occ_orig.size() * 4);
}
