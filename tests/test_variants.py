"""Runtime-compiled variants of fused element-wise struct-fors (host only:
generation and compilation need no device).

The generated kernel keeps each channel's value in registers from op to op:
a channel is loaded once per block (only when an op reads it before
anything writes it; the next block's loads are issued before this block's
stores) and stored once when written.  The device tests compare it with the interpreter bit for bit."""
import ctypes
import os
import re

import pytest

from paper_2012_08141_amd import _lib as L
from paper_2012_08141_amd import engine as E
from paper_2012_08141_amd.grid import SparseGrid


def prepare(tasks):
    arr = E._array(tasks)
    buf = ctypes.create_string_buffer(1 << 16)
    n = ctypes.c_size_t()
    st = L.lib().at_variant_prepare(arr, len(tasks), buf, len(buf), ctypes.byref(n))
    return st, buf.value.decode(), n.value


def loads_stores(src):
    """Channels loaded per block (the first block's loads) and stored."""
    loads = sorted(int(c) for c in re.findall(r"float4 p(\d+)a = \*reinterpret_cast<const float4 \*>", src))
    stores = sorted(int(c) for c in re.findall(r"\*reinterpret_cast<float4 \*>\(ch \+ (\d+)LL \* stride \+ off\) =", src))
    # every load has its prefetch for the next block and its second half
    for c in loads:
        assert ("float4 p%db = " % c) in src and ("float4 n%da = " % c) in src and ("float4 n%db = " % c) in src
    for c in stores:
        assert ("stride + off + 4) = c%db;" % c) in src
    return loads, stores


@pytest.fixture
def grid():
    return SparseGrid(64, 8, "bitmask", device=None)


def test_seed_program_compiles_with_one_load_and_store_per_channel(grid, private_caches):
    g = grid
    # the differentiation seed: grad_k = 0; lam = a_T; lam += a_T; lam += -2 target
    st, src, n = prepare([E.fill(g, [3], 0.0), E.copy(g, 1, 0), E.axpy(g, 1, 0, 1.0), E.axpy(g, 1, 2, -2.0)])
    assert st == L.AT_OK, L.lib().at_last_error()
    assert n == len(src) and "extern \"C\" __global__" in src
    loads, stores = loads_stores(src)
    assert loads == [0, 2] and stores == [1, 3]
    # the code object is in the disk cache
    d = os.path.join(private_caches, "atsparse", "variants")
    assert any(f.endswith(".co") for f in os.listdir(d))
    # a second prepare finds it (same source, no new file)
    before = set(os.listdir(d))
    assert prepare([E.fill(g, [3], 0.0), E.copy(g, 1, 0), E.axpy(g, 1, 0, 1.0), E.axpy(g, 1, 2, -2.0)])[0] == L.AT_OK
    assert set(os.listdir(d)) == before


def test_fill_array_and_chains(grid):
    g = grid
    st, src, _ = prepare([E.fill(g, [0], 7.0) for _ in range(10)])
    assert st == L.AT_OK
    assert loads_stores(src) == ([], [0])
    # chain_copy: y = x + 1, z = y + 4
    st, src, _ = prepare([E.copy(g, 1, 0), E.inc(g, 1, 1.0), E.copy(g, 2, 1), E.inc(g, 2, 4.0)])
    assert st == L.AT_OK
    assert loads_stores(src) == ([0], [1, 2])
    # normalise (m, mv -> v) then clearing m and mv: once it saves no memory
    # traffic (11 accesses per voxel either way) and stays on the
    # interpreter; twice over, the variant moves half the bytes
    one = [E.normalise(g, 0, 1, 4), E.fill(g, [0, 1, 2, 3], 0.0)]
    assert prepare(one)[0] == L.AT_E_UNSUPPORTED
    st, src, _ = prepare(one + one)
    assert st == L.AT_OK
    assert loads_stores(src) == ([0, 1, 2, 3], [0, 1, 2, 3, 4, 5, 6])
    # three copies move the same bytes as a variant: interpreter
    assert prepare([E.copy(g, 0, 5), E.copy(g, 1, 6), E.copy(g, 2, 7)])[0] == L.AT_E_UNSUPPORTED


def test_unsupported_programs(grid):
    g = grid
    assert prepare([E.jacobi(g, 0, 1, 2), E.copy(g, 0, 2)])[0] == L.AT_E_UNSUPPORTED
    assert prepare([E.copy(g, 0, 1)])[0] == L.AT_E_INVALID          # one task: no fusion
    other = SparseGrid(64, 8, "bitmask", device=None)
    assert prepare([E.copy(g, 0, 1), E.copy(other, 0, 1)])[0] == L.AT_E_UNSUPPORTED


@pytest.mark.parametrize("root", ["bitmask", "pointer"])
def test_tile_program_variant(root):
    """A fused advection node (two semi-Lagrangian ops sharing one Euler
    back-trace, a MacCormack correction, element-wise ops) compiles to a tile
    kernel with its ops written out: one back-trace computed once (the
    MacCormack op shares it), each op's channels and constants in the code,
    the root kind's lookup; an RK3 program stages the velocity tiles."""
    cap = 512 if root == "pointer" else 0
    g = SparseGrid(64, 10, root, cap, device=None)
    prog = [E.advect_sl(g, 0, 2, 7, 0.6), E.advect_sl(g, 1, 2, 8, 0.6), E.maccormack(g, 0, 2, 5, 6, 9, 0.6),
            E.copy(g, 5, 9), E.inc(g, 6, 0.25)]
    st, src, n = prepare(prog)
    assert st == L.AT_OK, L.lib().at_last_error()
    assert n == len(src) and 'void atst(' in src
    assert ("#define KIND %d" % (0 if root == "bitmask" else 1)) in src
    assert src.count("trace_tile(") == 2             # the helper and one shared back-trace
    assert "chan(g, 7)[off] = " in src and "chan(g, 8)[off] = " in src and "chan(g, 9)[off] = " in src
    assert "chan(g, 5)[off] = chan(g, 9)[off];" in src
    assert "chan(g, 6)[off] = chan(g, 6)[off] + 0x1p-2f;" in src
    assert "constexpr int NT = 2;" in src and "#define VOWN 1" in src
    # RK3 back-traces sample the velocity: three velocity tiles staged
    st, src, _ = prepare([E.advect_sl(g, 0, 2, 7, 0.6, rk3=True), E.advect_sl(g, 1, 2, 8, 0.6, rk3=True)])
    assert st == L.AT_OK
    assert "constexpr int NC = 5;" in src and "#define VOWN 0" in src and src.count("sample_staged(g, vs") == 2
    # two back-traces (different dt): two trace blocks
    st, src, _ = prepare([E.advect_sl(g, 0, 2, 7, 0.6), E.advect_sl(g, 1, 2, 8, -0.6)])
    assert st == L.AT_OK and src.count("trace_tile(") == 3


def test_tile_program_limits():
    """Which fused sampling nodes get a tile program: Euler back-traces by
    different velocities read each op's velocity at the voxel (no velocity
    staged); RK3 back-traces must share one velocity (its tiles are staged);
    at most four sampled fields are staged."""
    g = SparseGrid(64, 16, "bitmask", device=None)
    st, src, _ = prepare([E.advect_sl(g, 0, 2, 7, 0.5), E.advect_sl(g, 1, 10, 8, 0.5)])
    assert st == L.AT_OK and "#define V0 -1" in src and "#define VOWN 0" in src
    assert "chan(g, 10 + d)[off]" in src and "chan(g, 2 + d)[off]" in src
    st, _, _ = prepare([E.advect_sl(g, 0, 2, 7, 0.5, rk3=True), E.advect_sl(g, 1, 10, 8, 0.5, rk3=True)])
    assert st == L.AT_E_UNSUPPORTED
    four = [E.advect_sl(g, q, 5, 8 + q, 0.5) for q in range(4)]
    assert prepare(four)[0] == L.AT_OK
    five = four + [E.advect_sl(g, 4, 5, 12, 0.5)]
    assert prepare(five)[0] == L.AT_E_UNSUPPORTED


def test_variant_options():
    assert E.get_option(L.AT_OPTION_VARIANTS) == 0
    for m in (1, 2, 0):
        E.set_option(L.AT_OPTION_VARIANTS, m)
        assert E.get_option(L.AT_OPTION_VARIANTS) == m
    with pytest.raises(L.AtError):
        E.set_option(L.AT_OPTION_VARIANTS, 3)
    with pytest.raises(L.AtError):
        E.set_option(L.AT_OPTION_VARIANTS_LOADED, 1)
