"""CPU checks of the C ABI: the library loads, exports every entry point the
header declares, its struct layouts match the binding, and its host-side
logic (lambda schedules, free-energy estimators) agrees with the oracle.
No kernel is launched here."""
import ctypes as C
import os
import re
import subprocess

import numpy as np
import pytest

from oracle import estimators as OE
from paper_2201_04622_amd import eamfe as E

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "eamfe.h")


def declared_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^(?:int|double|const char\*)\s+(\w+)\(", text, flags=re.M)))


def test_library_exports_every_declared_symbol():
    L = E.lib()
    names = declared_functions()
    assert len(names) >= 20
    for n in names:
        assert hasattr(L, n), n
    out = subprocess.run(["nm", "-D", "--defined-only", E.LIB_PATH], capture_output=True, text=True).stdout
    exported = {l.split()[-1] for l in out.splitlines() if " T " in l}
    assert set(names) <= exported


def test_struct_layout_matches_header(tmp_path):
    src = tmp_path / "sz.c"
    src.write_text('#include "eamfe.h"\n#include <stdio.h>\n#include <stddef.h>\n'
                   'int main(void){printf("%zu %zu %zu %zu %zu\\n", sizeof(eamfe_replica), sizeof(eamfe_protocol),'
                   ' offsetof(eamfe_replica, seed), offsetof(eamfe_protocol, dt), offsetof(eamfe_protocol, skin));'
                   'return 0;}\n')
    exe = tmp_path / "sz"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    vals = [int(v) for v in subprocess.check_output([str(exe)]).split()]
    assert vals == [C.sizeof(E.Replica), C.sizeof(E.Protocol), E.Replica.seed.offset, E.Protocol.dt.offset,
                    E.Protocol.skin.offset]


def test_create_without_device_fails_cleanly():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    h = C.c_void_p()
    code = E.lib().eamfe_create(C.byref(h), 0, None, 0)
    assert code == 3 and not h.value       # EAMFE_EDEVICE


@pytest.mark.parametrize("mode,func,lf", [("fl", 2, 1.0), ("fl", 1, 1.0), ("hh", 2, 1.0), ("rs", 2, 0.0625),
                                          ("ein_rs", 2, 0.25)])
def test_lambda_schedule_matches_oracle(oracle_lib, mode, func, lf):
    p = E.protocol(mode, n_eq=37, n_sw=1000, n_hold=13, n_hold2=7, function=func, lambda_f=lf)
    lam = E.lambda_schedule(p)
    ref = oracle_lib.schedule(mode, 37, 1000, 13, 7, function=func, lambda_f=lf)
    assert lam.shape == ref.shape
    # the polynomial's terms reach 420 tau^6 before cancelling to O(1): ~1e-13 rounding
    assert np.abs(lam - ref).max() < 1e-12


def test_bad_protocols_rejected():
    with pytest.raises(E.EamfeError):
        E.lambda_schedule(E.protocol("fl", n_sw=0))
    with pytest.raises(E.EamfeError):
        E.lambda_schedule(E.protocol("rs", n_sw=10, lambda_f=0.0))
    with pytest.raises(E.EamfeError):
        E.lambda_schedule(E.protocol("fl", n_sw=10, function=3))


def test_estimators_match_oracle():
    rng = np.random.default_rng(0)
    for N, T, k, m in ((128, 100.0, 5.0, 55.845), (2000, 1400.0, 3.0, 55.845), (11664, 100.0, 5.787, 55.845)):
        assert E.einstein_free_energy(N, T, k, m) == pytest.approx(OE.einstein_free_energy(N, T, k, m), rel=1e-14)
        V = N / 0.0859
        assert E.fixed_cm_correction(N, V, T, k) == pytest.approx(OE.fixed_cm_correction(N, V, T, k), rel=1e-13)
        Wf = rng.normal(1.2, 0.05, 10)
        Wb = rng.normal(-1.1, 0.05, 10)
        got = E.fl_free_energy(Wf, Wb, N, T, k, m, N, V)
        ref = OE.frenkel_ladd(Wf, Wb, N, T, k, m, N, V)
        assert np.allclose(got, ref, rtol=1e-12, atol=1e-14)


def test_rs_estimator_matches_oracle():
    rng = np.random.default_rng(1)
    p = E.protocol("rs", n_eq=50, n_sw=400, n_hold=30, n_hold2=20, lambda_f=0.0625)
    S = 50 + 800 + 30 + 20
    W = np.cumsum(rng.normal(0.0, 0.3, S))
    T = np.arange(100.0, 1601.0, 1.0)
    got = E.rs_free_energy(p, W, -4.2, 100.0, 127, T)
    fw, bw = OE.rs_work_curves(W, 50, 400, 30)
    ref = OE.reversible_scaling(-4.2, 100.0, 0.0625, 127, fw, bw, T)
    assert np.abs(got - ref).max() < 1e-10
