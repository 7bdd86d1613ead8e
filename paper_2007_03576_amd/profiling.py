"""Kernel-class timing read from libhqr (HIP events recorded by the driver on
the stream each kernel is launched on) and the roofline summary of bench.py."""
import ctypes

from ._lib import lib

CLASSES = ["lds_iteration", "chase_windows", "update_gemm", "large_aed", "other"]
KERNELS = {"lds_iteration": "k_iter", "chase_windows": "k_chase", "update_gemm": "k_update_s/k_gemm64",
           "large_aed": "k_corner_deflate/k_restore_global", "other": "k_fin_*/k_find_block"}
FP64_PEAK_TFLOPS = 78.6   # MI355X dense FP64 (matrix and vector)
HBM_PEAK_GBS = 8000.0


def enable(on: bool) -> None:
    lib().hqr_profile_enable(1 if on else 0)


def reset() -> None:
    lib().hqr_profile_reset()


def read() -> dict:
    n = len(CLASSES)
    ms = (ctypes.c_double * n)()
    cnt = (ctypes.c_int64 * n)()
    fl = (ctypes.c_double * n)()
    by = (ctypes.c_double * n)()
    lib().hqr_profile_read(ms, cnt, fl, by, n)
    return {c: {"ms": ms[i], "launches": int(cnt[i]), "flops": fl[i], "bytes": by[i]}
            for i, c in enumerate(CLASSES)}


def lds_split() -> dict:
    """Fractions of the LDS iteration kernel's device time spent in the Schur
    solve, the reordering and the Hessenberg restoration, with the event
    counts behind them (chase phases, single-bulge steps, swaps, launches of
    each kind) and the device clock cycles per phase and per swap."""
    t = (ctypes.c_int64 * 10)()
    lib().hqr_profile_ticks(t, 10)
    tot = max(int(t[3]), 1)
    out = {"schur": t[0] / tot, "reorder": t[1] / tot, "restore": t[2] / tot,
           "phases": int(t[4]), "bulge_steps": int(t[5]), "swaps": int(t[6]),
           "small_launches": int(t[7]), "aed_launches": int(t[8]), "reorder_phases": int(t[9])}
    # wall clock at 100 MHz, shader clock 2.4 GHz
    if t[4] > 0:
        out["us_per_phase"] = t[0] / 100.0 / t[4]
    if t[6] > 0:
        out["us_per_swap"] = t[1] / 100.0 / t[6]
    if t[9] > 0:
        out["us_per_reorder_phase"] = t[1] / 100.0 / t[9]
    return out


def summary(prof: dict, steps: int) -> dict:
    return {c: {"ms_per_step": v["ms"] / max(steps, 1), "launches_per_step": v["launches"] / max(steps, 1),
                "kernel": KERNELS[c]} for c, v in prof.items()}


def _entry(prof: dict, cls: str, steps: int) -> dict:
    g = prof[cls]
    bound = "mfma" if cls == "update_gemm" else "alu"
    out = {"bound": bound, "achieved": None, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": None,
           "traffic": None, "kernel": KERNELS[cls], "class": cls}
    if g["launches"] == 0 or g["ms"] <= 0:
        return out
    avg_s = g["ms"] / g["launches"] / 1e3
    fpl = g["flops"] / g["launches"]
    ach = fpl / avg_s / 1e12
    out.update({"achieved": ach, "frac": ach / FP64_PEAK_TFLOPS, "avg_launch_us": avg_s * 1e6,
                "flops_per_launch": fpl, "bytes_per_launch": g["bytes"] / g["launches"],
                "launches_per_step": g["launches"] / max(steps, 1), "ms_per_step": g["ms"] / max(steps, 1)})
    if bound == "alu":
        # one workgroup runs on one of the 256 CUs: its own ceiling is 1/256 of the chip
        out["peak_one_cu"] = FP64_PEAK_TFLOPS / 256.0
        out["frac_one_cu"] = ach / (FP64_PEAK_TFLOPS / 256.0)
    return out


def roofline(prof: dict, steps: int) -> dict:
    """Roofline entry of the dominant kernel class by time (counted algorithmic
    flops per launch / average launch duration vs the FP64 peak), with the
    FP64-MFMA update kernel reported alongside."""
    dom = max(prof, key=lambda c: prof[c]["ms"])
    out = _entry(prof, dom, steps)
    out["mfma_update"] = _entry(prof, "update_gemm", steps)
    return out
