"""The host stages (partition, weld) and the C ABI's argument checks under
AddressSanitizer and UndefinedBehaviorSanitizer: the host sources are rebuilt
instrumented (paper_1903_12359_amd.build.build_sanitized), and the host-only
tests of the C ABI run in a child process that loads that build with the ASan
runtime preloaded.  Any report of either sanitizer ends the child with its
own exit code, which fails this test; no device call is made."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_host_code_is_clean_under_asan_and_ubsan():
    from paper_1903_12359_amd import build as b
    try:
        lib = b.build_sanitized(verbose=False)
        env = b.sanitizer_env()
    except (RuntimeError, subprocess.CalledProcessError, OSError) as e:   # no hipcc in this checkout
        pytest.skip(f"sanitizer build unavailable: {e}")
    env["PGCP_LIB"] = lib
    env["PYTHONPATH"] = ROOT + os.pathsep + env.get("PYTHONPATH", "")
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_abi_host.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    out = r.stdout + r.stderr
    assert "AddressSanitizer" not in out and "runtime error:" not in out, out[-4000:]
    assert r.returncode == 0, out[-4000:]
    assert " passed" in out


def test_build_rejects_a_streaming_kernel_with_scratch():
    """The build's resource check (compiler remarks) refuses a streaming CG
    kernel that spills: its persistent grid could not be guaranteed resident."""
    from paper_1903_12359_amd import build as b
    head = "device.hip:1:1: remark: Function Name: _ZN4pgcp12k_pcg_streamIdLi256EEEvNS_6CGArgsIT_EE\n"
    b._check_scratch(head + "device.hip:1:1: remark:     ScratchSize [bytes/lane]: 0\n")
    other = "device.hip:1:1: remark: Function Name: _ZN4pgcp5k_pcgIdLi256ELi6EEEvNS_6CGArgsIT_EE\n"
    b._check_scratch(other + "device.hip:1:1: remark:     ScratchSize [bytes/lane]: 276\n")
    with pytest.raises(RuntimeError):
        b._check_scratch(head + "device.hip:1:1: remark:     ScratchSize [bytes/lane]: 12\n")
