"""Top-level oracle entry point: run a scheme in original or fundamental form.

``run`` mirrors what the library's ``fdtd_run`` computes: physical fields at
integer time levels on entry and on return, the scheme's input processing once
at the start and its output processing once at the end (Table I, "Input" and
"Output" rows), and optionally the trace of the conserved energy of the main
iteration state.
"""
from __future__ import annotations

from . import conventional, crank_nicolson, fundamental
from .yee import Grid, clean

SCHEMES = ("adi", "lod1", "ss2", "lod2")
FORMS = ("fundamental", "conventional")
# D'Yakonov and Douglas-Gunn splittings of Sec. II-E (their original forms
# take no nonhomogeneous term; the fundamental forms take the ADI convention)
SPLITTINGS = ("dy", "dg")
# Crank-Nicolson without factorization (Sec. II-E), a global sparse solve per step
UNFACTORIZED = ("cn",)


def run(scheme: str, form: str, g: Grid, fields, steps: int, source=None,
        energy_every: int = 0):
    """Advance `fields` (six node arrays, [k, j, i]) by `steps` full time steps.

    Returns (fields_out, trace) where trace lists the scheme's invariant energy
    (see ``conventional.invariant``) at steps 0, e, 2e, ... (e = energy_every;
    empty if 0).  Tangential E on the walls is treated as 0 on input.
    """
    if (scheme not in SCHEMES + SPLITTINGS + UNFACTORIZED) or form not in FORMS:
        raise ValueError((scheme, form))
    if scheme == "cn":
        return crank_nicolson.run_fields(g, fields, steps, form, energy_every, source)
    u = clean(fields, g)
    trace = []

    def record(n, value_fn):
        if energy_every and n % energy_every == 0:
            trace.append(value_fn())

    if scheme in SPLITTINGS:
        # both splittings give the ADI fields u^n; their invariant is ADI's,
        # W((1/2 I + dt/4 B) u^n)
        if source is not None and form == "conventional":
            raise ValueError("the original D'Yakonov and Douglas-Gunn splittings take no source")

        def rec(n, un):
            record(n, lambda: conventional.invariant("adi", un, g))

        if form == "conventional":
            rec(0, u)
            for n in range(steps):
                u = conventional.splitting_step(scheme, u, g)
                rec(n + 1, u)
            return u, trace
        run_f = fundamental.dyakonov if scheme == "dy" else fundamental.douglas_gunn
        return run_f(u, g, steps, rec, source), trace

    if form == "conventional":
        u = conventional.input_processing(scheme, u, g)
        record(0, lambda: conventional.invariant(scheme, u, g))
        for n in range(steps):
            u = conventional.step(scheme, u, g, n, source)
            record(n + 1, lambda: conventional.invariant(scheme, u, g))
        return conventional.output_processing(scheme, u, g), trace

    if scheme == "adi":
        st = fundamental.FundamentalADI(u, g)
        record(0, st.invariant)
        for n in range(steps):
            st.step(source)
            record(n + 1, st.invariant)
        return st.fields(), trace

    from .yee import energy
    if scheme == "lod2":
        u = fundamental.lod2_input(u, g)
    record(0, lambda: energy(u, g))
    for n in range(steps):
        u = fundamental.lod_step(scheme, u, g, n, source)
        record(n + 1, lambda: energy(u, g))
    if scheme == "lod2":
        u = fundamental.lod2_output(u, g)
    return u, trace
