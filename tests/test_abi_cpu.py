"""CPU-side checks of the C ABI: the library loads, exports every symbol that
include/swf.h declares, and its host-side validation rejects bad inputs with
the documented status codes (swf_workspace_size runs no device code)."""
import ctypes as C
import os
import re

import pytest

import swf_workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def S():
    from paper_2512_16889_amd import swf
    return swf


def header_symbols():
    txt = open(os.path.join(ROOT, "include", "swf.h")).read()
    return sorted(set(re.findall(r"\b(swf_[a-z_]+)\s*\(", txt)))


def test_exports_every_declared_symbol(S):
    syms = header_symbols()
    assert "swf_init" in syms and "swf_step" in syms and "swf_amplitude" in syms
    for s in syms:
        assert hasattr(S._lib, s), s
    assert set(syms) == set(S.EXPORTED)


def test_supported_sizes(S):
    for n in (16, 32, 48, 64, 80, 128, 256, 320, 384, 512, 768, 1024):
        assert S.supported_n(n)
    for n in (8, 100, 2048, 1000):
        assert not S.supported_n(n)


def wsize(S, prob, prec=0):
    grids, terms, ffirst, solves, verts, win = S.marshal(prob)
    opt = S.Options()
    opt.prec = prec
    out = C.c_size_t(0)
    code = S._lib.swf_workspace_size(grids, len(prob.grids), terms, ffirst, len(prob.fields), solves,
                                     len(prob.solves), verts, len(prob.vertices), C.byref(win), C.byref(opt),
                                     C.byref(out))
    return code, out.value, S._lib.swf_last_error(None).decode()


def test_workspace_size_scales_with_state(S):
    a = W.config_2d(n=64, n_solves=4, steps=10)
    code, b64, _ = wsize(S, a, 0)
    assert code == 0
    code, b32, _ = wsize(S, a, 1)
    assert code == 0
    state64 = 4 * 4 * 64 * 64 * 16 * 4
    assert b64 >= state64 and b32 >= state64 // 2 and b64 > b32


def test_validation_errors(S):
    base = W.config_2d(n=64, L=160.0, n_solves=1, steps=10)
    assert wsize(S, base)[0] == 0
    bad = W.config_2d(n=100, n_solves=1, steps=10)
    assert wsize(S, bad)[0] == S.SWF_E_UNSUPPORTED
    nyq = W.config_2d(n=64, L=160.0, n_solves=1, steps=10)
    nyq.solves[0].p = [5.0, 0.0, 0.0]          # beyond pi n / L = 1.26
    code, _, msg = wsize(S, nyq)
    assert code == S.SWF_E_ARG and "Nyquist" in msg
    unstable = W.config_2d(n=64, L=160.0, dt=2.5, n_solves=1, steps=10)
    code, _, msg = wsize(S, unstable)
    assert code == S.SWF_E_ARG and "stability" in msg
    triv = W.config_1d(n=64, L=100.0, steps=10)
    triv.fields[0][0].fx[1] = W.gauss(3.0)      # depends on trivial axis y
    code, _, msg = wsize(S, triv)
    assert code == S.SWF_E_ARG and "trivial" in msg
    win = W.config_1d(n=64, L=100.0, steps=10)
    win.window = W.Window(0.0, 1.0, 0.3)
    assert wsize(S, win)[0] == S.SWF_E_ARG
    bwbad = W.config_bw_1d(n=64, L=100.0, steps=4)
    bwbad.vertices[0].k = [0.0, 1.0, 0.0]       # p2 + q2 = 1.2 != 1.0
    code, _, msg = wsize(S, bwbad)
    assert code == S.SWF_E_ARG and "p + q" in msg
    kinds = W.config_bw_1d(n=64, L=100.0, steps=4)
    kinds.vertices[0].u_solve, kinds.vertices[0].v_solve = 1, 0
    assert wsize(S, kinds)[0] == S.SWF_E_ARG


def test_packet_validation(S):
    k, eps = [0.0, 1.2, 0.0], [-1.0, 0.0, 0.0]

    def packet(modes):
        prob = W.config_bw_1d(n=64, L=100.0, steps=4)
        vx = prob.vertices[0]
        k0 = [0.0, vx.k[1], 0.0]
        prob.vertices = [W.Vertex(vx.u_solve, vx.v_solve, vx.k, vx.eps, [(k0 if m[0] is None else m[0], m[1], m[2])
                                                                         for m in modes])]
        return prob
    assert wsize(S, packet([(None, eps, 0.5), (None, eps, 0.5)]))[0] == 0
    assert wsize(S, packet([(None, eps, 1.0 / 65)] * 65))[0] == S.SWF_E_ARG
    code, _, msg = wsize(S, packet([(None, eps, 0.5), ([0.1, 0.7, 0.0], eps, 0.5)]))
    assert code == S.SWF_E_ARG and "trivial" in msg
    code, _, msg = wsize(S, packet([(None, eps, complex(float("nan"), 0.0))]))
    assert code == S.SWF_E_ARG and "finite" in msg
    code, _, msg = wsize(S, packet([(None, eps, 1.0), ([0.0, 0.0, 0.0], eps, 0.0)]))
    assert code == S.SWF_E_ARG and "non-zero" in msg
    grids, terms, ffirst, solves, verts, win = S.marshal(packet([(None, eps, 1.0)]))
    opt = S.Options()
    opt.bw_partial = 1
    out = C.c_size_t(0)
    assert S._lib.swf_workspace_size(grids, 1, terms, ffirst, 1, solves, 2, verts, 1, C.byref(win), C.byref(opt),
                                     C.byref(out)) == S.SWF_E_UNSUPPORTED


def test_in_state_validation(S):
    prob = W.config_1d(n=64, L=100.0, steps=10)
    prob.solves = [W.Solve(W.U_IN, 1, prob.solves[0].p), W.Solve(W.V_IN, -1, prob.solves[0].p)]
    assert wsize(S, prob)[0] == 0
    prob.solves[1].kind = W.V_OUT                   # opposite time directions in one context
    code, _, msg = wsize(S, prob)
    assert code == S.SWF_E_UNSUPPORTED and "in- and out-states" in msg
    prob.solves[1].kind = 4
    assert wsize(S, prob)[0] == S.SWF_E_ARG


def test_stepper_validation(S):
    import dataclasses
    prob = W.config_bw_1d(n=64, L=100.0, steps=4)
    w = prob.window
    prob = dataclasses.replace(prob, window=W.Window(w.t_in, w.t_out, w.dt, "dp5"))
    grids, terms, ffirst, solves, verts, win = S.marshal(prob)

    def size(**kw):
        opt = S.Options()
        for k, v in kw.items():
            setattr(opt, k, v)
        out = C.c_size_t(0)
        code = S._lib.swf_workspace_size(grids, 1, terms, ffirst, 1, solves, 2, verts, 1, C.byref(win), C.byref(opt),
                                         C.byref(out))
        return code, out.value
    c4, b4 = size(stepper=S.SWF_RK4)
    c5, b5 = size(stepper=S.SWF_DP5)
    assert c4 == 0 and c5 == 0 and b5 > b4            # eight state arrays per solve instead of four
    assert size(stepper=S.SWF_DP5, bw_partial=1)[0] == S.SWF_E_UNSUPPORTED
    cip, bip = size(stepper=S.SWF_IPRK4)
    assert cip == 0 and b4 < bip < b5                 # six state arrays per solve
    assert size(stepper=S.SWF_IPRK4, bw_partial=1)[0] == S.SWF_E_UNSUPPORTED
    assert size(stepper=7)[0] == S.SWF_E_ARG
    assert S.workspace_size(prob) == b5               # the binding takes the stepper from the window
