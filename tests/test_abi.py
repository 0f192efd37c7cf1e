"""The C ABI on the CPU: libvqmc.so loads, exports every entry point that
include/vqmc.h declares, and rejects bad arguments before touching a GPU."""
import ctypes as ct
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", f) for f in sorted(os.listdir(os.path.join(ROOT, "include")))
           if f.endswith(".h")]

V = pytest.importorskip("paper_2108_13830_amd.vqmc")

if not os.path.exists(V.LIB_PATH):
    pytest.skip("libvqmc.so not built", allow_module_level=True)


def declared():
    """Every function declared in include/*.h (comments stripped)."""
    names = set()
    for h in HEADERS:
        text = re.sub(r"/\*.*?\*/", "", open(h).read(), flags=re.S)
        names |= set(re.findall(r"\b(vqmc_[a-z0-9_]+)\s*\(", text))
    return sorted(names)


def test_every_declared_symbol_is_exported():
    names = declared()
    assert len(names) == 15
    lib = ct.CDLL(V.LIB_PATH)
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    # and the binding knows every one of them, with the same names
    assert sorted(n for n, _, _ in V.SIGNATURES) == names


def test_num_params_and_model_validation():
    assert V.num_params(V.Model(4, 4, 2)) == 336
    assert V.num_params(V.Model(10, 16, 6)) == 14080
    assert V.num_params(V.Model(24, 32, 8)) == 74304
    for bad in (V.Model(5, 4, 2), V.Model(26, 4, 2), V.Model(4, 12, 2), V.Model(4, 4, 0),
                V.Model(4, 4, 2, eloc=3),
                V.Model(4, 4, 2, prec=V.PREC_BF16), V.Model(4, 8, 2, prec=7), V.Model(4, 8, 2, marshall=2),
                V.Model(4, 4, 2, symmetry=2)):
        assert V.num_params(bad) == -1


def test_status_strings():
    lib = V.lib()
    for code in range(8):
        assert lib.vqmc_status_string(code)
    assert lib.vqmc_status_string(99) == b"unknown status"


def test_argument_errors_need_no_gpu():
    lib = V.lib()
    bad = V.Model(5, 4, 2).c()
    good = V.Model(4, 4, 2).c()
    nul = ct.c_void_p(0)
    assert lib.vqmc_log_psi(ct.byref(bad), nul, nul, 1, nul, nul, nul) == 1
    assert lib.vqmc_local_energy(ct.byref(bad), nul, nul, 1, nul, nul, nul, 0, nul) == 1
    assert lib.vqmc_local_energy_noalloc(ct.byref(bad), nul, nul, 1, nul, nul, nul) == 1
    # the allocation-free form: dense only, no symmetrisation, checked arguments
    sym = V.Model(4, 4, 2, symmetry=1).c()
    lc = V.Model(16, 16, 2, eloc=V.ELOC_LIGHTCONE).c()
    assert lib.vqmc_local_energy_noalloc(ct.byref(sym), nul, nul, 1, nul, nul, nul) == 1
    assert lib.vqmc_local_energy_noalloc(ct.byref(lc), nul, nul, 1, nul, nul, nul) == 1
    assert lib.vqmc_local_energy_noalloc(ct.byref(good), nul, nul, -1, nul, nul, nul) == 2
    assert lib.vqmc_local_energy_noalloc(ct.byref(good), nul, nul, 3, nul, nul, nul) == 1
    assert lib.vqmc_log_psi(ct.byref(good), nul, nul, -1, nul, nul, nul) == 2
    assert lib.vqmc_log_psi(ct.byref(good), nul, nul, 3, nul, nul, nul) == 1
    # B = 0 is a valid empty call: nothing is launched
    assert lib.vqmc_log_psi(ct.byref(good), nul, nul, 0, nul, nul, nul) == 0
    assert lib.vqmc_local_energy(ct.byref(good), nul, nul, 0, nul, nul, nul, 0, nul) == 0
    # the light-cone evaluation needs 16 or 32 channels and a workspace
    lc = V.Model(16, 32, 8, eloc=V.ELOC_LIGHTCONE).c()
    n = ct.c_size_t(0)
    assert lib.vqmc_local_energy_workspace(ct.byref(lc), 64, ct.byref(n)) == 0 and n.value > 0
    assert lib.vqmc_local_energy(ct.byref(lc), ct.c_void_p(8), ct.c_void_p(8), 64, ct.c_void_p(8), nul,
                                 nul, 0, nul) == 4
    lc4 = V.Model(16, 4, 2, eloc=V.ELOC_LIGHTCONE).c()
    assert lib.vqmc_local_energy_workspace(ct.byref(lc4), 64, ct.byref(n)) == 1
    # the method a model resolves to
    meth = ct.c_int32(-1)
    assert lib.vqmc_local_energy_method(ct.byref(lc), ct.byref(meth)) == 0 and meth.value == V.ELOC_LIGHTCONE
    auto24 = V.Model(24, 32, 8).c()
    assert lib.vqmc_local_energy_method(ct.byref(auto24), ct.byref(meth)) == 0 and meth.value == V.ELOC_LIGHTCONE
    auto10 = V.Model(10, 16, 6).c()
    assert lib.vqmc_local_energy_method(ct.byref(auto10), ct.byref(meth)) == 0 and meth.value == V.ELOC_DENSE
    assert lib.vqmc_local_energy_method(ct.byref(lc4), ct.byref(meth)) == 1
    # the light cone keeps the boxes of distance 1 .. n in two LDS buffers: at
    # 24 x 24 the split-BF16 and FP32 forms fit n <= 8 (the dense evaluation
    # is used beyond), the single-BF16 form any n
    for prec, n_layers, want in ((V.PREC_BF16X3, 8, V.ELOC_LIGHTCONE), (V.PREC_BF16X3, 9, V.ELOC_DENSE),
                                 (V.PREC_FP32, 9, V.ELOC_DENSE), (V.PREC_BF16, 16, V.ELOC_LIGHTCONE)):
        mm = V.Model(24, 32, n_layers, prec=prec).c()
        assert lib.vqmc_local_energy_method(ct.byref(mm), ct.byref(meth)) == 0 and meth.value == want
    forced = V.Model(24, 32, 9, prec=V.PREC_BF16X3, eloc=V.ELOC_LIGHTCONE).c()
    assert lib.vqmc_local_energy_method(ct.byref(forced), ct.byref(meth)) == 1
    assert lib.vqmc_local_energy_workspace(ct.byref(forced), 64, ct.byref(n)) == 1
    # 16 x 16 fits every depth in every form
    deep16 = V.Model(16, 32, 16, prec=V.PREC_BF16X3, eloc=V.ELOC_LIGHTCONE).c()
    assert lib.vqmc_local_energy_method(ct.byref(deep16), ct.byref(meth)) == 0 and meth.value == V.ELOC_LIGHTCONE
    # dense: room for the packed weights of the 8 layers (36 KiB each), optional
    dense = V.Model(16, 32, 8, eloc=V.ELOC_DENSE).c()
    assert lib.vqmc_local_energy_workspace(ct.byref(dense), 64, ct.byref(n)) == 0 and n.value == 8 * 36864
    # the symmetrised local energy needs a workspace for its 4B rotated copies
    sym = V.Model(10, 16, 6, eloc=V.ELOC_DENSE, symmetry=1).c()
    assert lib.vqmc_local_energy_workspace(ct.byref(sym), 64, ct.byref(n)) == 0
    assert n.value >= 4 * 64 * 100 + 4 * 64 * (8 + 8 + 4)
    assert lib.vqmc_local_energy(ct.byref(sym), ct.c_void_p(8), ct.c_void_p(8), 64, ct.c_void_p(8), nul,
                                 nul, 0, nul) == 4
    assert lib.vqmc_local_energy(ct.byref(sym), nul, nul, 0, nul, nul, nul, 0, nul) == 0
    symlc = V.Model(16, 32, 8, eloc=V.ELOC_LIGHTCONE, symmetry=1).c()
    m = ct.c_size_t(0)
    assert lib.vqmc_local_energy_workspace(ct.byref(lc), 256, ct.byref(n)) == 0
    assert lib.vqmc_local_energy_workspace(ct.byref(symlc), 64, ct.byref(m)) == 0 and m.value > n.value
    # a 24 x 24 lattice does not fit the 512-row engine of C <= 16 (dense and sampler)
    big16 = V.Model(24, 16, 2, eloc=V.ELOC_DENSE).c()
    assert lib.vqmc_log_psi(ct.byref(big16), ct.c_void_p(8), ct.c_void_p(8), 1, ct.c_void_p(8), nul, nul) == 2
    assert lib.vqmc_sample(ct.byref(big16), ct.c_void_p(8), ct.c_void_p(8), nul, 1, 1, 0, 0, 0, nul, nul) == 2
    assert lib.vqmc_sample(ct.byref(good), nul, nul, nul, 2, 1, 0, 0, 5, nul, nul) == 1
    assert lib.vqmc_sample(ct.byref(good), nul, nul, nul, 0, 1, 0, 0, 0, nul, nul) == 0
    n = ct.c_size_t(0)
    assert lib.vqmc_log_derivs_workspace(ct.byref(good), 16, ct.byref(n)) == 0 and n.value > 0
    assert lib.vqmc_log_derivs(ct.byref(good), nul, nul, 16, nul, 10, nul, 0, nul) == 2  # ldO < P
    assert lib.vqmc_log_derivs(ct.byref(good), nul, nul, 16, ct.c_void_p(8), 336, ct.c_void_p(8),
                               0, nul) in (1, 4)


def test_sr_argument_errors_and_workspace():
    lib = V.lib()
    n = ct.c_size_t(0)
    ok = V.SrOpts().c()
    # auto: the smaller exact form
    assert lib.vqmc_sr_workspace(4096, 14080, ct.byref(ok), ct.byref(n)) == 0
    assert 4096 * 4096 * 8 <= n.value < 14080 * 14080 * 8  # the sample-space matrix
    assert lib.vqmc_sr_workspace(20000, 14080, ct.byref(ok), ct.byref(n)) == 0
    assert n.value >= 14080 * 14080 * 8  # the explicit S matrix
    ch = V.SrOpts(method=V.SR_CHOLESKY).c()
    assert lib.vqmc_sr_workspace(4096, 14080, ct.byref(ch), ct.byref(n)) == 0
    assert n.value >= 14080 * 14080 * 8
    cg = V.SrOpts(method=V.SR_CG).c()
    assert lib.vqmc_sr_workspace(16384, 74304, ct.byref(cg), ct.byref(n)) == 0
    assert n.value < 74304 * 74304 * 8 // 100  # matrix-free
    bad = V.SrOpts(eps=0.0).c()
    assert lib.vqmc_sr_workspace(10, 10, ct.byref(bad), ct.byref(n)) == 1
    assert lib.vqmc_sr_workspace(1, 10, ct.byref(ok), ct.byref(n)) == 2
    nul = ct.c_void_p(0)
    assert lib.vqmc_sr_solve(nul, 10, nul, 10, 10, ct.byref(ok), nul, nul, nul, 0, None, nul) == 1
    assert lib.vqmc_sr_solve(ct.c_void_p(8), 5, ct.c_void_p(8), 10, 10, ct.byref(ok), ct.c_void_p(8),
                             nul, nul, 0, None, nul) == 2
    assert lib.vqmc_sr_solve(ct.c_void_p(8), 10, ct.c_void_p(8), 10, 10, ct.byref(ok), ct.c_void_p(8),
                             nul, nul, 0, None, nul) == 4
