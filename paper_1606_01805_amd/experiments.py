"""The paper's own experiments at full scale, run through the library.

  transport  Sec. 3: neutrally buoyant circles, ellipses (AR 2), squares and
             triangles released at rest at y0/H = 0.25, 0.5, 0.75 in the
             Re = 20 Couette channel of 10 L x 4 L (L = 100), the AR-10
             rectangle released at 0.25, and the circle released at 0.25
             with an initial x velocity of 0.125 and 0.25 u_wall; all as
             channels of one batched handle.  Records the particle state every
             `every` steps and the x velocity along the vertical line through
             each centroid at t u_wall / L = 10, 50 and 500 (the local slip
             profiles of Sec. 3.2).
  refine     Sec. 2.1: the circle settling in the closed 4 N x 30 N box at
             N = 20, 40, 80 and 160 points per diameter, terminal Re = 0.1
             (gravity from the wall-corrected Stokes drag, see
             workloads.configs.paper_sedimentation_circle), density ratio
             1.2, tau = 1; terminal velocity per N (mesh refinement study).
  kernels    Sec. 2.2: the ellipse (AR 2, L = 100) settling from (2 L, 24 L)
             with theta0 = pi/4, Re = 12.5, Fr = 0.126, density ratio 1.1, with
             each of the five interpolation kernels (Eqs. (10), (17)-(20)) as
             channels of one handle.

Each run writes a compressed .npz of raw series; `summarize_*` turn them into
the quantities the paper prints.  Every step of the method runs in the HIP
library; this module only drives it and reduces its recorded outputs.

  python -m paper_1606_01805_amd.experiments transport|refine|kernels OUT_DIR
"""
import json
import math
import os
import sys
import time

import numpy as np

from workloads import configs as C

TRANSPORT_CASES = ([(f, y, 0.0) for f in ("circle", "ellipse", "square", "triangle") for y in (0.25, 0.5, 0.75)]
                   + [("rectangle", 0.25, 0.0), ("circle", 0.25, 0.125), ("circle", 0.25, 0.25)])
PROFILE_TIMES = (10.0, 50.0, 500.0)  # t u_wall / L of the slip profiles


def _log(*a):
    print(*a, flush=True)


def run_transport(out_dir, L=100, t_end=500.0, every=500, storage=C.STORE_F32, cases=TRANSPORT_CASES,
                  tuning=None):
    from . import Solver

    wl = C.paper_couette(cases, L=L, storage=storage)
    cfg0 = wl.channels[0][0]
    uw = cfg0["u_wall"][3][0]
    steps_per_t = L / uw
    n_steps = int(round(t_end * steps_per_t))
    prof_steps = sorted(int(round(t * steps_per_t)) for t in PROFILE_TIMES if t <= t_end)
    s = Solver(wl.channels, tuning=tuning)
    rec, times, profiles = [], [], {}
    done, t0 = 0, time.time()
    marks = sorted(set(list(range(every, n_steps + 1, every)) + prof_steps))
    for m in marks:
        s.step(m - done, record=False)
        done = m
        if m % every == 0:
            rec.append(s.particles())
            times.append(m)
        if m in prof_steps:
            cols = []
            pst = s.particles()
            for ch in range(len(wl.channels)):
                _, ux, _ = s.fields(ch)
                xc = int(round(pst[ch, 0])) % cfg0["nx"]
                cols.append(ux[:, xc])
            profiles[m] = np.array(cols)
        if m % (every * 200) == 0 or m == n_steps:
            _log(f"transport: {m}/{n_steps} steps, {time.time() - t0:.0f} s")
    s.close()
    out = os.path.join(out_dir, f"transport_L{L}.npz")
    np.savez_compressed(out, steps=np.array(times), rec=np.array(rec),
                        profile_steps=np.array(sorted(profiles)),
                        profiles=np.array([profiles[k] for k in sorted(profiles)]),
                        cases=json.dumps(cases), L=L, u_wall=uw, H=cfg0["ny"] - 1, nx=cfg0["nx"],
                        storage=storage)
    _log("wrote", out)
    return out


def run_refine(out_dir, Ns=(20, 40, 80, 160), t_visc=80.0, every=None, storage=C.STORE_F32):
    """Each resolution runs t_visc N^2 steps: about eight times the slowest
    viscous time across the channel, 16 N^2 nu^-1 / pi^2 = 9.7 N^2 steps."""
    from . import Solver

    res = {}
    for N in Ns:
        ch, u_inf = C.paper_sedimentation_circle(N, storage=storage)
        n_steps = int(t_visc * N * N)
        ev = every or max(1, n_steps // 2000)
        s = Solver([ch])
        t0 = time.time()
        rec, times, done = [], [], 0
        while done < n_steps:
            k = min(ev, n_steps - done)
            s.step(k, record=False)
            done += k
            rec.append(s.particles()[0])
            times.append(done)
            if len(times) % 200 == 0:
                _log(f"refine N={N}: {done}/{n_steps} steps, {time.time() - t0:.0f} s")
        s.close()
        res[N] = dict(steps=np.array(times), rec=np.array(rec), u_inf=u_inf)
        _log(f"refine N={N}: done, v_y = {rec[-1][4]:.6e} (u_inf {u_inf:.6e})")
    out = os.path.join(out_dir, "refine.npz")
    np.savez_compressed(out, Ns=np.array(Ns), **{f"steps_{N}": res[N]["steps"] for N in Ns},
                        **{f"rec_{N}": res[N]["rec"] for N in Ns}, **{f"uinf_{N}": res[N]["u_inf"] for N in Ns},
                        storage=storage)
    _log("wrote", out)
    return out


def run_kernels(out_dir, L=100, n_steps=40000, every=100, storage=C.STORE_F64):
    from . import Solver

    chans, u = [], None
    for k in range(5):
        ch, u = C.paper_sedimentation_ellipse(k, L=L, storage=storage)
        chans.append(ch)
    s = Solver(chans)
    rec, times, done, t0 = [], [], 0, time.time()
    while done < n_steps:
        s.step(every, record=False)
        done += every
        rec.append(s.particles())
        times.append(done)
        if done % (every * 50) == 0:
            _log(f"kernels: {done}/{n_steps} steps, {time.time() - t0:.0f} s")
    s.close()
    out = os.path.join(out_dir, f"kernels_L{L}.npz")
    np.savez_compressed(out, steps=np.array(times), rec=np.array(rec), L=L, u=u, storage=storage)
    _log("wrote", out)
    return out


# ---------------------------------------------------------------------------
# Reductions to the quantities the paper prints.
# ---------------------------------------------------------------------------

def _period_and_amplitude(t, w):
    """Mean, half peak-to-peak amplitude and mean period (from upward
    crossings of the mean) of a periodic series w(t)."""
    m = float(w.mean())
    amp = float((w.max() - w.min()) / 2)
    z = np.where((w[:-1] < m) & (w[1:] >= m))[0]
    if len(z) < 2:
        return m, amp, float("nan")
    tz = t[z] + (m - w[z]) / (w[z + 1] - w[z]) * (t[z + 1] - t[z])
    return m, amp, float(np.diff(tz).mean())


def summarize_transport(path, tail=0.2):
    d = np.load(path)
    cases = [tuple(c) for c in json.loads(str(d["cases"]))]
    L, uw, H = float(d["L"]), float(d["u_wall"]), float(d["H"])
    t = d["steps"] * uw / L                      # t u_wall / L
    rec = d["rec"]                               # [samples, channels, 10]
    gam = uw / H                                 # shear rate of the undisturbed flow
    n = len(t)
    tailsl = slice(int((1 - tail) * n), n)
    rows = []
    for ch, (fam, y0, u0) in enumerate(cases):
        y = rec[:, ch, 1] / H
        ux = rec[:, ch, 3] / uw
        om = rec[:, ch, 5]
        ush = uw * rec[:, ch, 1] / H             # undisturbed Couette velocity at the centroid
        row = dict(family=fam, y0=y0, u0=u0,
                   y_eq=float(y[tailsl].mean()), y_osc=float((y[tailsl].max() - y[tailsl].min()) / 2),
                   ux_eq=float(ux[tailsl].mean()),
                   omega_eq_L_over_u=float(-om[tailsl].mean() * L / uw),
                   omega_slip_over_gamma=float((om[tailsl] + 0.5 * gam).mean() / gam),
                   u_slip_first=float((rec[0, ch, 3] - ush[0]) / uw),
                   u_slip_final=float((rec[-1, ch, 3] - ush[-1]) / uw))
        if fam in ("square", "rectangle", "ellipse", "triangle"):
            half = slice(n // 2, n)
            m, amp, per = _period_and_amplitude(t[half], -om[half] * L / uw)
            row.update(omega_mean=m, omega_amplitude=amp, omega_period=per)
        rows.append(row)
    # trajectories of the circle released at 0.25 with different initial velocities
    base = [i for i, c in enumerate(cases) if c == ("circle", 0.25, 0.0)]
    spread = None
    if base:
        b = base[0]
        others = [i for i, c in enumerate(cases) if c[0] == "circle" and c[1] == 0.25 and c[2] != 0.0]
        if others:
            spread = {str(cases[i][2]): float(np.abs(rec[:, i, 1] - rec[:, b, 1]).max() / H) for i in others}
    prof = {}
    if "profiles" in d and len(d["profile_steps"]):
        yy = np.arange(int(H) + 1)
        ush = uw * yy / H
        for k, st in enumerate(d["profile_steps"]):
            for ch, c in enumerate(cases):
                if c in (("circle", 0.25, 0.0), ("circle", 0.75, 0.0)):
                    slip = (ush - d["profiles"][k, ch]) / uw
                    prof[f"{c[0]}@{c[1]} t={st * uw / L:g}"] = dict(
                        max=float(slip.max()), min=float(slip.min()),
                        y_of_max=float(yy[int(slip.argmax())] / H), y_of_min=float(yy[int(slip.argmin())] / H))
    return dict(t_end=float(t[-1]), rows=rows, u0_spread=spread, slip_profiles=prof)


def summarize_refine(path):
    d = np.load(path)
    Ns = [int(n) for n in d["Ns"]]
    vt = {}
    for N in Ns:
        rec = d[f"rec_{N}"]
        v = -rec[:, 4]
        # terminal velocity: the mean over the last 5 % of the run, with the
        # change over the last 10 % as its settling indicator
        k = max(1, len(v) // 20)
        vt[N] = dict(v_terminal=float(v[-k:].mean()), u_inf=float(d[f"uinf_{N}"]),
                     last10_change=float(abs(v[-1] - v[int(0.9 * len(v))]) / v[-1]),
                     re_terminal=float(v[-k:].mean() * N / ((1.0 - 0.5) / 3.0)))
    ref = Ns[-1]
    for N in Ns:
        vt[N]["v_over_u_inf"] = vt[N]["v_terminal"] / vt[N]["u_inf"]
    for N in Ns[:-1]:
        vt[N]["rel_error_vs_finest"] = abs(vt[N]["v_over_u_inf"] - vt[ref]["v_over_u_inf"]) / vt[ref]["v_over_u_inf"]
    orders = {}
    for a, b in zip(Ns[:-2], Ns[1:-1]):
        ea, eb = vt[a]["rel_error_vs_finest"], vt[b]["rel_error_vs_finest"]
        orders[f"{a}->{b}"] = math.log(ea / eb) / math.log(b / a)
    # order from three successive resolutions, free of the finest one's own
    # error: p = log2((v_a - v_b) / (v_b - v_c)) for N_c = 2 N_b = 4 N_a
    rich = {}
    for a, b, c in zip(Ns[:-2], Ns[1:-1], Ns[2:]):
        va, vb, vc = (vt[n]["v_over_u_inf"] for n in (a, b, c))
        rich[f"{a},{b},{c}"] = math.log(abs(va - vb) / abs(vb - vc)) / math.log(b / a)
    return dict(resolutions=vt, observed_order_vs_finest=orders, observed_order_three_levels=rich)


def summarize_kernels(path, y_probe=18.0):
    d = np.load(path)
    L = float(d["L"])
    rec = d["rec"]
    names = ["exponential", "cubic", "quartic", "cosine", "polynomial"]
    y = rec[:, :, 1] / L
    th = rec[:, :, 2] / math.pi
    out = {"y_final_over_L": {names[k]: float(y[-1, k]) for k in range(5)}}
    # theta/pi of each kernel at the height y/L = y_probe, interpolated along
    # each trajectory, and its difference from the exponential kernel
    at = {}
    for k in range(5):
        yk, tk = y[:, k], th[:, k]
        i = np.where((yk[:-1] >= y_probe) & (yk[1:] < y_probe))[0]
        if len(i):
            i = i[0]
            f = (y_probe - yk[i]) / (yk[i + 1] - yk[i])
            at[names[k]] = float(tk[i] + f * (tk[i + 1] - tk[i]))
    out[f"theta_over_pi_at_y{y_probe:g}L"] = at
    if "exponential" in at:
        out["rel_diff_vs_exponential_at_probe"] = {n: abs(v - at["exponential"]) / abs(at["exponential"])
                                                   for n, v in at.items() if n != "exponential"}
    out["max_abs_theta_over_pi_diff_vs_exponential"] = {
        names[k]: float(np.abs(th[:, k] - th[:, 0]).max()) for k in range(1, 5)}
    out["theta_over_pi_final"] = {names[k]: float(th[-1, k]) for k in range(5)}
    return out


def main(argv):
    what, out_dir = argv[1], argv[2]
    os.makedirs(out_dir, exist_ok=True)
    if what == "transport":
        p = run_transport(out_dir)
        print(json.dumps(summarize_transport(p)))
    elif what == "refine":
        p = run_refine(out_dir)
        print(json.dumps(summarize_refine(p)))
    elif what == "kernels":
        p = run_kernels(out_dir)
        print(json.dumps(summarize_kernels(p)))
    else:
        raise SystemExit(f"unknown experiment {what}")


if __name__ == "__main__":
    main(sys.argv)
