"""Host-side checks of the C ABI that need no GPU: the library loads, every
entry point declared in include/ile.h is exported, the binding's struct
layouts and integer constants equal the C ones, and calls fail cleanly
without a device."""
import ctypes as C
import os
import re
import subprocess

import pytest

import paper_2505_11655_amd as ile

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ile.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:ile_status|void|size_t|const char \*)\s*\*?\s*(ile_\w+)\s*\(", src, flags=re.M)
    return sorted(set(names))


def test_library_exports_every_declared_symbol():
    if not os.path.exists(ile.LIB_PATH):
        pytest.skip("libile.so not built")
    names = declared_functions()
    assert len(names) >= 20
    lib = C.CDLL(ile.LIB_PATH)
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    # the binding covers every declared entry point
    assert set(names) <= set(ile.EXPORTS)


def test_struct_layouts_match_header(tmp_path):
    """Compile a probe against ile.h with gcc and compare sizes and offsets."""
    probe = tmp_path / "probe.c"
    structs = {"ile_problem": ile.ile_problem, "ile_prior": ile.ile_prior, "ile_marg": ile.ile_marg,
               "ile_job_info": ile.ile_job_info, "ile_gmm_params": ile.ile_gmm_params,
               "ile_gmm_opts": ile.ile_gmm_opts, "ile_server_opts": ile.ile_server_opts,
               "ile_job_opts": ile.ile_job_opts, "ile_result": ile.ile_result, "ile_av_opts": ile.ile_av_opts,
               "ile_av_state": ile.ile_av_state, "ile_qv_shape": ile.ile_qv_shape}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "ile.h"', "int main(void){"]
    for name, cls in structs.items():
        lines.append(f'printf("{name} %zu\\n", sizeof({name}));')
        for f, _ in cls._fields_:
            lines.append(f'printf("{name}.{f} %zu\\n", offsetof({name}, {f}));')
    lines.append("return 0;}")
    probe.write_text("\n".join(lines))
    exe = tmp_path / "probe"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), str(probe), "-o", str(exe)])
    out = subprocess.check_output([str(exe)]).decode().split("\n")
    got = dict(l.rsplit(" ", 1) for l in out if l.strip())
    for name, cls in structs.items():
        assert int(got[name]) == C.sizeof(cls), name
        for f, _ in cls._fields_:
            assert int(got[f"{name}.{f}"]) == getattr(cls, f).offset, f"{name}.{f}"


def test_constants_match_header():
    """Every integer #define of ile.h that the binding also names has the
    header's value (flags, integrators, pool and overlap routes...)."""
    src = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    defs = dict(re.findall(r"^#define\s+(ILE_\w+)\s+(\d+)u?\s*$", src, flags=re.M))
    shared = [k for k in defs if hasattr(ile, k)]
    assert {"ILE_QV_AUTO", "ILE_QV_DIRECT", "ILE_QV_DECIMATED", "ILE_POOL_MIXTURE", "ILE_INT_AC"} <= set(shared)
    for k in shared:
        assert getattr(ile, k) == int(defs[k]), k


def test_no_device_is_a_clean_error():
    if not os.path.exists(ile.LIB_PATH):
        pytest.skip("libile.so not built")
    try:
        import torch
        if torch.cuda.is_available():
            pytest.skip("a GPU is present")
    except ImportError:
        pass
    with pytest.raises(ile.IleError) as e:
        ile.ile_ctx_create(0, 0)
    assert e.value.status == -4
    assert "device" in ile.ile_last_error().lower()
    # null handles are rejected, not dereferenced
    st = ile.lib().ile_eval_lnL(None, 10, None, 10, None, None, None, None)
    assert st == -1
    st = ile.lib().ile_marginalize(None, 0, None, 1, None, None)
    assert st == -1
