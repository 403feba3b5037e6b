"""Invariants of the host packer (owner-computes slot layout, lane-major
records, chunk bounds), built with g++ from the library's sources."""
import ctypes
import os
import subprocess

import numpy as np
import pytest

from paper_1402_2626_amd import synth

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(os.path.dirname(HERE), "paper_1402_2626_amd", "csrc")


@pytest.fixture(scope="module")
def lib(tmp_path_factory):
    out = tmp_path_factory.mktemp("pack") / "libpack_host.so"
    subprocess.run(["g++", "-O2", "-std=c++17", "-shared", "-fPIC", os.path.join(HERE, "pack_host.cpp"),
                    os.path.join(SRC, "packer.cpp"), "-o", str(out)], check=True)
    lib = ctypes.CDLL(str(out))
    lib.pe_test_pack_msg.restype = ctypes.c_char_p
    return lib


def pack(lib, s, seg, max_slots=1152):
    arrs = [np.ascontiguousarray(a) for a in (s.poly_ptr, s.mon_ptr, s.var_idx, s.exps, s.coef)]
    sizes = np.zeros(9, np.int64)
    st = lib.pe_test_pack(s.level, s.n_vars, s.n_polys, *[ctypes.c_void_p(a.ctypes.data) for a in arrs],
                          seg, max_slots, ctypes.c_void_p(sizes.ctypes.data))
    assert st == 0, lib.pe_test_pack_msg()
    nch, nocc, ncol, M = int(sizes[0]), int(sizes[1]), int(sizes[2]), int(sizes[3])
    chunks = np.zeros((nch, 9), np.int64)
    occ = np.zeros((nocc, 4), np.uint16)
    colptr = np.zeros(ncol, np.uint16)
    mmeta = np.zeros(M, np.uint32)
    mcoef = np.zeros(M * 2 * s.level)
    cptr = np.zeros(s.n_polys + 1, np.uint32)
    lib.pe_test_pack_get(*[ctypes.c_void_p(a.ctypes.data) for a in (chunks, occ, colptr, mmeta, mcoef, cptr)])
    rowdesc = np.zeros((s.n_polys * 4, 9), np.int64)
    assert lib.pe_test_pack_rowdesc(ctypes.c_void_p(rowdesc.ctypes.data)) == 4
    return dict(chunks=chunks, occ=occ, colptr=colptr, mmeta=mmeta, mcoef=mcoef, chunk_ptr=cptr, rowdesc=rowdesc,
                n=int(sizes[4]), max_slots_used=int(sizes[5]))


def check_rowdesc(P, n_polys):
    # row p's first four chunk descriptors in row order, empty (count 0) past the row's last chunk
    for p in range(n_polys):
        c0, c1 = int(P["chunk_ptr"][p]), int(P["chunk_ptr"][p + 1])
        for j in range(4):
            got = P["rowdesc"][p * 4 + j]
            if c0 + j < c1:
                assert np.array_equal(got, P["chunks"][c0 + j])
            else:
                assert got[4] == 0


def lanes_for(k, seg):
    need = (k + seg - 1) // seg
    s = 1
    while s < need:
        s <<= 1
    return s


@pytest.mark.parametrize("seg", [2, 4, 8])
def test_pack_invariants(lib, seg):
    s = synth.random_system(7, 2, n_vars=60, n_polys=9, m=70, k=11, exp_lo=1, exp_hi=4)
    # mixed sizes: add monomials of other lengths to one polynomial
    polys = []
    for p in range(s.n_polys):
        mons = []
        for t in range(int(s.poly_ptr[p]), int(s.poly_ptr[p + 1])):
            vs, ds = s.monomial(t)
            mons.append((0, list(zip(vs.tolist(), ds.tolist()))))
        polys.append(mons)
    rng = synth.rng_for(8)
    for k in (0, 1, 3, 31, 40):
        vs = np.sort(rng.choice(60, size=k, replace=False))
        polys[2].append((0, [(int(v), 2) for v in vs]))
    polys.append([])  # empty polynomial
    coef = synth.unit_circle(rng, sum(len(m) for m in polys), 2)
    s = synth.from_monomial_lists(2, 60, polys, coef_limbs=coef)
    P = pack(lib, s, seg)
    n = P["n"]
    assert n == 60
    seen_mon = set()
    for p in range(s.n_polys):
        # monomials of polynomial p, as multisets of (var, exp)
        want = sorted(tuple(sorted(zip(*[a.tolist() for a in s.monomial(t)])))
                      for t in range(int(s.poly_ptr[p]), int(s.poly_ptr[p + 1])))
        got = []
        for ch in range(int(P["chunk_ptr"][p]), int(P["chunk_ptr"][p + 1])):
            ob, mb, cb, poly, count, nslots, width, sl, segc = P["chunks"][ch]
            assert poly == p and width == count * sl and sl <= 64 and segc <= seg
            assert nslots + 1 <= P["max_slots_used"]
            cp = P["colptr"][cb:cb + n + 1].astype(int)
            assert cp[0] == 0 and cp[-1] == nslots and np.all(np.diff(cp) >= 0)
            col_of_slot = np.repeat(np.arange(n), np.diff(cp))
            slots = []
            for g in range(count):
                k = int(P["mmeta"][mb + g])
                assert lanes_for(max(k, 1), seg) <= sl and k <= sl * segc
                occs = [None] * k
                base, extra = k // sl, k % sl
                for q in range(sl):
                    ln = base + (1 if q < extra else 0)
                    for i in range(segc):
                        var, ex, slot, _ = P["occ"][ob + i * width + g * sl + q]
                        if i >= ln:
                            # neutral padding: the constant-1 column, exponent 1, the dummy slot
                            assert (var, ex, slot) == (n, 1, nslots)
                            continue
                        occs[q + i * sl] = (int(var), int(ex))  # lane q holds occurrences q, q + s, ...
                        assert col_of_slot[slot] == var
                        slots.append(int(slot))
                assert None not in occs
                assert [v for v, _ in occs] == sorted(v for v, _ in occs)  # canonical order
                got.append(tuple(occs))
                seen_mon.add(mb + g)
            assert sorted(slots) == list(range(nslots)), "slots must be a permutation"
            # within a column, slots follow (monomial, position) order
            for c in range(n):
                seg_slots = list(range(cp[c], cp[c + 1]))
                assert seg_slots == sorted(seg_slots)
        assert sorted(got) == want
    assert len(seen_mon) == s.n_monomials
    check_rowdesc(P, s.n_polys)


def test_chunk_budget(lib):
    s = synth.random_system(9, 4, n_vars=300, n_polys=2, m=500, k=20, exp_lo=1, exp_hi=2)
    P = pack(lib, s, 4, max_slots=1100)
    assert P["max_slots_used"] <= 1100
    assert np.all(P["chunks"][:, 5] + 1 <= 1100)
    assert np.all(P["chunks"][:, 6] <= 256)
    check_rowdesc(P, s.n_polys)


def test_packer_under_sanitizers(tmp_path):
    """The validator and packer, built with g++ and the address and
    undefined-behaviour sanitizers, over random and malformed systems."""
    exe = tmp_path / "pack_fuzz"
    build = subprocess.run(["g++", "-O1", "-g", "-std=c++17", "-fsanitize=address,undefined",
                            "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
                            os.path.join(HERE, "pack_fuzz.cpp"), os.path.join(SRC, "packer.cpp"), "-o", str(exe)],
                           capture_output=True, text=True)
    assert build.returncode == 0, build.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1", UBSAN_OPTIONS="print_stacktrace=1")
    env.pop("LD_PRELOAD", None)
    run = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=600)
    assert run.returncode == 0 and run.stdout.strip().endswith("OK"), run.stdout[-2000:] + run.stderr[-4000:]


def _orig_maps(lib, P, M):
    mon = np.zeros(M, np.uint32)
    occ = np.zeros(P["occ"].shape[0], np.uint32)
    lib.pe_test_pack_orig(ctypes.c_void_p(mon.ctypes.data), ctypes.c_void_p(occ.ctypes.data))
    return mon, occ


@pytest.mark.parametrize("seg", [2, 4, 8])
def test_pack_input_order_maps(lib, seg):
    """The maps behind the per-monomial output: every input monomial appears
    once among the packed monomials; every record's input occurrence names
    the record's variable and exponent and lies in its monomial's input
    range; neutral records map to no occurrence; every occurrence is named
    exactly once (variables shuffled within monomials)."""
    s = synth.random_system(21, 2, n_vars=50, n_polys=7, m=30, k=9, exp_lo=1, exp_hi=4)
    rng = synth.rng_for(22)
    perm = np.concatenate([rng.permutation(np.arange(a, b)) for a, b in zip(s.mon_ptr[:-1], s.mon_ptr[1:])])
    s.var_idx = np.ascontiguousarray(s.var_idx[perm])
    s.exps = np.ascontiguousarray(s.exps[perm])
    P = pack(lib, s, seg)
    mon, occ = _orig_maps(lib, P, s.n_monomials)
    assert sorted(mon.tolist()) == list(range(s.n_monomials))
    seen = np.zeros(s.nnz, np.int64)
    for ch in P["chunks"]:
        occ_base, mon_base, _, _, count, nslots, width, lanes, segc = (int(v) for v in ch)
        for i in range(segc):
            for lam in range(width):
                r = occ_base + i * width + lam
                o = int(occ[r])
                var, ex, slot = int(P["occ"][r][0]), int(P["occ"][r][1]), int(P["occ"][r][2])
                if slot == nslots:
                    assert o == 0xFFFFFFFF
                    continue
                t = int(mon[mon_base + lam // lanes])
                assert s.mon_ptr[t] <= o < s.mon_ptr[t + 1]
                assert int(s.var_idx[o]) == var and int(s.exps[o]) == ex
                seen[o] += 1
    assert np.all(seen == 1)


def test_pack_real_coefficients(lib):
    """A real system (level 8 | L) packs one component per coefficient: the
    packed coefficients are the input's limbs in packed monomial order."""
    s = synth.random_system(23, 2, n_vars=20, n_polys=5, m=9, k=4)
    coef_real = np.ascontiguousarray(s.coef[:1])
    arrs = [np.ascontiguousarray(a) for a in (s.poly_ptr, s.mon_ptr, s.var_idx, s.exps, coef_real)]
    sizes = np.zeros(9, np.int64)
    st = lib.pe_test_pack(8 | 2, s.n_vars, s.n_polys, *[ctypes.c_void_p(a.ctypes.data) for a in arrs], 4, 1152,
                          ctypes.c_void_p(sizes.ctypes.data))
    assert st == 0, lib.pe_test_pack_msg()
    nch, nocc, ncol, M = int(sizes[0]), int(sizes[1]), int(sizes[2]), int(sizes[3])
    chunks = np.zeros((nch, 9), np.int64)
    occ = np.zeros((nocc, 4), np.uint16)
    colptr = np.zeros(ncol, np.uint16)
    mmeta = np.zeros(M, np.uint32)
    mcoef = np.zeros(M * 2 * 2)  # room for the complex layout; a real one fills half
    cptr = np.zeros(s.n_polys + 1, np.uint32)
    lib.pe_test_pack_get(*[ctypes.c_void_p(a.ctypes.data) for a in (chunks, occ, colptr, mmeta, mcoef, cptr)])
    mon, _ = _orig_maps(lib, dict(occ=occ), M)
    for tp in range(M):
        t = int(mon[tp])
        assert np.array_equal(mcoef[2 * tp:2 * tp + 2], s.coef[0, :, t])
    assert np.all(mcoef[2 * M:] == 0.0)
    # an invalid level code is refused
    st = lib.pe_test_pack(16 | 2, s.n_vars, s.n_polys, *[ctypes.c_void_p(a.ctypes.data) for a in arrs], 4, 1152,
                          ctypes.c_void_p(sizes.ctypes.data))
    assert st == -1
