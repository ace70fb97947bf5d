"""CPU checks of the C-ABI boundary: the built library exports every function that
include/d4dgs.h declares, the binding mirrors the header's structs, and host-side
argument checks reject bad sizes without touching a GPU."""
import ctypes as C
import os
import re
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "d4dgs.h")
LIB = os.path.join(ROOT, "paper_2503_22159_amd", "libd4dgs.so")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(d4dgs_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_function():
    names = declared_functions()
    assert len(names) >= 14, names
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True, check=True).stdout
    exported = set(re.findall(r"\bT (d4dgs_\w+)", out))
    missing = [n for n in names if n not in exported]
    assert not missing, missing


def test_library_holds_gfx950_code():
    out = subprocess.run(["strings", LIB], capture_output=True, text=True, check=True).stdout
    assert "gfx950" in out


def test_binding_structs_match_header_sizes():
    from paper_2503_22159_amd import binding as B

    # sizes implied by the header's field lists (LP64)
    assert C.sizeof(B.Camera) == 4 * 2 + 4 * 7 + 4 * 9 + 4 * 3 + 4 * 3
    assert C.sizeof(B.Scene) == 8 + 8 * 8
    assert C.sizeof(B.Splats) == 8 + 8 * 5 + 8  # capacity (padded), 5 pointers, motion (padded)
    assert C.sizeof(B.Bins) == 8 + 8 * 5
    assert B.lib.d4dgs_abi_version() == B.ABI_VERSION
    assert set(B.EXPORTS) == set(declared_functions())


def test_host_argument_checks():
    from paper_2503_22159_amd import binding as B

    b = C.c_size_t(0)
    assert B.lib.d4dgs_workspace_size(100, 0, 10, 1000, C.byref(b)) == B.ERR_INVALID_ARG
    assert B.lib.d4dgs_workspace_size(100, 64, 64, 0, C.byref(b)) == B.ERR_INVALID_ARG
    assert B.lib.d4dgs_workspace_size(100, 64, 64, 1000, C.byref(b)) == B.OK and b.value > 1000 * 16
    assert B.lib.d4dgs_project(None, None, 0.0, None, None, None) == B.ERR_INVALID_ARG
    assert "NULL" in B.last_error()
    s = B.Scene()
    s.n, s.sh_degree = 10, 5
    cam = B.Camera()
    assert B.lib.d4dgs_project(C.byref(s), C.byref(cam), 0.0, None, None, None) == B.ERR_INVALID_ARG
    assert B.lib.d4dgs_serve_create(None, None, None) == B.ERR_INVALID_ARG
    # the fused projection + binning and the workspace initialisation check their
    # arguments before touching the device
    need = B.workspace_size(10, 64, 64, 1000)
    assert B.lib.d4dgs_workspace_init(None, need, 10, 64, 64, 1000, None) == B.ERR_INVALID_ARG
    assert B.lib.d4dgs_workspace_init(C.c_void_p(256), need, 10, 0, 64, 1000, None) == B.ERR_INVALID_ARG
    assert B.lib.d4dgs_workspace_init(C.c_void_p(256), need, 10, 64, 64, 0, None) == B.ERR_INVALID_ARG
    # a workspace smaller than d4dgs_workspace_size gives for these sizes
    assert B.lib.d4dgs_workspace_init(C.c_void_p(256), need - 1, 10, 64, 64, 1000, None) == B.ERR_INVALID_ARG
    assert b"workspace_bytes" in B.lib.d4dgs_last_error()
    assert B.lib.d4dgs_project_bin(None, None, 0.0, None, None, None, 0, None, None, None) == B.ERR_INVALID_ARG
    s.n, s.sh_degree = 0, 0
    assert B.lib.d4dgs_project_bin(C.byref(s), C.byref(cam), 0.0, None, None, None, 0, None, None,
                                   None) == B.ERR_INVALID_ARG  # an all-zero camera


def test_camera_checks_reject_bad_cameras():
    """The camera checks (shared by d4dgs_project and the server's submit) run on the host
    before any GPU work: non-finite or non-positive fields and image sizes beyond what the
    kernels index are rejected with INVALID_ARG and a message."""
    import math

    from paper_2503_22159_amd import binding as B
    from paper_2503_22159_amd import inputs

    s = B.Scene()
    s.n, s.sh_degree = 0, 0
    good = inputs.look_at((0.0, 0.0, -6.0), width=64, height=48)

    def project(mutate):
        cam = B.camera_struct(good)
        mutate(cam)
        return B.lib.d4dgs_project(C.byref(s), C.byref(cam), 0.5, None, None, None)

    # a good camera passes the camera checks and stops at the missing splats
    assert project(lambda c: None) == B.ERR_INVALID_ARG and "splats" in B.last_error()
    cases = [
        (lambda c: setattr(c, "width", 0), "size"),
        (lambda c: setattr(c, "height", 65535 * 16 + 1), "size"),
        # each side within 65535 tiles, but more tiles than a launch grid can index
        (lambda c: (setattr(c, "width", 65535 * 16), setattr(c, "height", 65535 * 16)), "size"),
        (lambda c: setattr(c, "fx", 0.0), "intrinsics"),
        (lambda c: setattr(c, "cy", math.nan), "intrinsics"),
        (lambda c: setattr(c, "tan_fovy", -1.0), "field of view"),
        (lambda c: setattr(c, "znear", 0.0), "znear"),
        (lambda c: c.R.__setitem__(4, math.inf), "rotation"),
        (lambda c: c.campos.__setitem__(1, math.nan), "position"),
    ]
    for mutate, word in cases:
        assert project(mutate) == B.ERR_INVALID_ARG, word
        assert word in B.last_error(), (word, B.last_error())
    b = C.c_size_t(0)
    assert B.lib.d4dgs_workspace_size(10, 65535 * 16, 65535 * 16, 1000, C.byref(b)) == B.ERR_INVALID_ARG
