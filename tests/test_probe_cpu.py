"""CPU-side checks of the measurement library libgpf_probe.so (kept out of the
radiance library's ABI): it loads, exports the FMA-ceiling probe and the
operand-form probe, and both reject bad arguments on the host before any
launch (no GPU is touched by these calls)."""
import ctypes
import os

from paper_2512_12459_amd import probe

FAKE = ctypes.c_void_p(0x1000)   # never dereferenced: every call below fails validation


def _lib():
    assert os.path.exists(probe.PROBE_PATH), "build the probe library first"
    return probe._load()


def test_probe_library_exports_both_probes():
    lib = ctypes.CDLL(probe.PROBE_PATH)
    assert hasattr(lib, "gpf_probe_valu")
    assert hasattr(lib, "gpf_probe_valu_form")


def test_ceiling_probe_rejects_bad_arguments():
    lib = _lib()
    assert lib.gpf_probe_valu(None, 256, 1, 1, None) == 1          # no output buffer
    assert lib.gpf_probe_valu(FAKE, 256, 0, 1, None) == 1          # no workgroups
    assert lib.gpf_probe_valu(FAKE, 256, 1, 0, None) == 1          # no iterations
    assert lib.gpf_probe_valu(FAKE, 255, 1, 1, None) == 1          # output shorter than 256 floats


def test_form_probe_rejects_unknown_forms_and_bad_sizes():
    lib = _lib()
    for form in (-1, 5, 1000):
        assert lib.gpf_probe_valu_form(FAKE, 256, 1, 1, form, 1.0, 0.0, None) == 1
    assert lib.gpf_probe_valu_form(FAKE, 511, 2, 1, 0, 1.0, 0.0, None) == 1
    assert lib.gpf_probe_valu_form(None, 256, 1, 1, 0, 1.0, 0.0, None) == 1
    assert set(probe.FORMS) == {0, 1, 2, 3, 4}
