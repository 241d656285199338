"""CPU checks of the C ABI: the library loads and exports every declared symbol, and the
host-only defaults agree with the binding and the oracle's parameters."""
import ctypes as C
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = []
    for h in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if h.endswith(".h"):
            src = open(os.path.join(ROOT, "include", h)).read()
            src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
            names += re.findall(r"\b(comet_[a-z0-9_]+)\s*\(", src)
    return sorted(set(names))


def test_library_exports_every_declared_symbol():
    from paper_2609_21803_amd import native
    L = C.CDLL(native.LIB_PATH)
    names = declared_functions()
    assert "comet_evaluate" in names and "comet_create" in names
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing


def test_default_params_agree_with_binding_and_oracle():
    import oracle
    from paper_2609_21803_amd import native
    lib_defaults = native.SolverParams.library_defaults()
    assert lib_defaults == native.SolverParams()
    o = oracle.Params()
    for f in ("al_max", "gn_max", "chol_retries", "ls_trials", "max_rejects", "mu0", "mu_min", "rho0", "rho_min",
              "rho_max", "armijo_c1", "eta_star", "omega_star", "rc_star", "eps_feas", "mu0_warm"):
        assert getattr(o, f) == getattr(lib_defaults, f), f
    assert (lib_defaults.ref_al_max, lib_defaults.ref_gn_max) == (oracle.REFINE["al_max"], oracle.REFINE["gn_max"])


def test_product_does_not_import_the_oracle():
    pkg = os.path.join(ROOT, "paper_2609_21803_amd")
    for dp, _, fs in os.walk(pkg):
        for f in fs:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                src = open(os.path.join(dp, f)).read()
                assert "import oracle" not in src and "from oracle" not in src and "comet_oracle" not in src, f


def test_struct_layouts_match_the_header(tmp_path):
    """Field offsets and sizes of the parameter structs: C compiler on include/comet.h vs
    the binding's ctypes structures."""
    import subprocess
    from paper_2609_21803_amd import native
    structs = {"comet_expand_params": native.ExpandParamsC, "comet_solver_params": native.SolverParamsC,
               "comet_expand_stats": native.ExpandStatsC}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "comet.h"', 'int main(void) {']
    for s, cls in structs.items():
        lines.append(f'  printf("{s} size %zu\\n", sizeof({s}));')
        for f, _ in cls._fields_:
            lines.append(f'  printf("{s} {f} %zu\\n", offsetof({s}, {f}));')
    lines.append("  return 0;\n}")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(src)])
    out = subprocess.check_output([str(exe)], text=True).split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l.strip()}
    for s, cls in structs.items():
        assert got[(s, "size")] == C.sizeof(cls), s
        for f, _ in cls._fields_:
            assert got[(s, f)] == getattr(cls, f).offset, (s, f)


def test_network_hooks_check_scalars_and_accept_an_empty_batch_on_the_host():
    """The network hooks reject bad scalar arguments and treat B = 0 as a no-op with NULL
    arrays, all before any device call (so this runs without a GPU)."""
    from paper_2609_21803_amd import native
    L = C.CDLL(native.LIB_PATH)
    P, I32, I64 = C.c_void_p, C.c_int32, C.c_int64
    L.comet_mlp_encode.argtypes = [C.c_int, P, I64, P, P, P, P, P, P, I32, I32, P]
    L.comet_mlp_targets.argtypes = [C.c_int, P, I64, P, I32, P, P, I32, P, P, P, P, P, P]
    L.comet_mlp_decode_warm.argtypes = [C.c_int, P, I64, P, I32, P, P, P, P, I32, I32, P]
    L.comet_mlp_forward.argtypes = [P, P, I64, P, P]
    OK, EINVAL = 0, -1
    enc = lambda task, B, smax=6, in_dim=416: L.comet_mlp_encode(task, None, B, *([None] * 6), smax, in_dim, None)
    tgt = lambda task, B, nmax=24, smax=6: L.comet_mlp_targets(task, None, B, None, nmax, None, None, smax,
                                                               *([None] * 6))
    dec = lambda task, B, out_dim=736, nmax=24: L.comet_mlp_decode_warm(task, None, B, None, out_dim, *([None] * 4),
                                                                        6, nmax, None)
    for task in (native.TASK_PUSH, native.TASK_FLIP, native.TASK_PUSH_TIMED):
        assert enc(task, 0) == OK and tgt(task, 0) == OK and dec(task, 0) == OK
        assert enc(task, -1) == EINVAL and tgt(task, -1) == EINVAL and dec(task, -1) == EINVAL
        assert enc(task, 0, smax=7) == EINVAL and enc(task, 0, in_dim=399) == EINVAL
        assert tgt(task, 0, nmax=0) == EINVAL and dec(task, 0, out_dim=721) == EINVAL
        assert enc(task, 4) == EINVAL and tgt(task, 4) == EINVAL and dec(task, 4) == EINVAL   # NULL arrays
    for task in (native.TASK_PUSH_FREE, native.TASK_PUSH_FREE_TIMED):   # eight segments, wider blocks
        assert enc(task, 0, smax=8, in_dim=528) == OK and tgt(task, 0, smax=8) == OK
        assert dec(task, 0, out_dim=962) == OK
        assert enc(task, 0, smax=9, in_dim=528) == EINVAL and enc(task, 0, smax=8, in_dim=527) == EINVAL
        assert tgt(task, 0, smax=9) == EINVAL and dec(task, 0, out_dim=961) == EINVAL
        assert enc(task, 4, smax=8, in_dim=528) == EINVAL and dec(task, 4, out_dim=962) == EINVAL
    assert enc(5, 0) == EINVAL and tgt(5, 0) == EINVAL and dec(5, 0) == EINVAL              # unknown task
    assert L.comet_mlp_forward(None, None, 0, None, None) == EINVAL                          # no network
