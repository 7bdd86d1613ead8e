"""Kernel-class timing read from libhqr (HIP events recorded by the driver on
the stream each kernel is launched on) and the roofline summary of bench.py."""
import ctypes

from ._lib import lib

CLASSES = ["lds_iteration", "chase_windows", "update_gemm", "large_aed", "other"]
KERNELS = {"lds_iteration": "k_iter", "chase_windows": "k_chase", "update_gemm": "k_update",
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


def summary(prof: dict, steps: int) -> dict:
    return {c: {"ms_per_step": v["ms"] / max(steps, 1), "launches_per_step": v["launches"] / max(steps, 1),
                "kernel": KERNELS[c]} for c, v in prof.items()}


def roofline(prof: dict, steps: int) -> dict:
    """Roofline entry for the update products (the FP64-MFMA kernel): counted
    algorithmic flops per launch / average launch duration, against the FP64
    matrix peak; the dominant class by time is reported alongside."""
    dom = max(prof, key=lambda c: prof[c]["ms"])
    g = prof["update_gemm"]
    if g["launches"] == 0 or g["ms"] <= 0:
        return {"bound": "mfma", "achieved": None, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": None,
                "traffic": None, "kernel": "k_update", "dominant_class": dom}
    avg_s = g["ms"] / g["launches"] / 1e3
    flops_per_launch = g["flops"] / g["launches"]
    ach = flops_per_launch / avg_s / 1e12
    return {"bound": "mfma", "achieved": ach, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
            "frac": ach / FP64_PEAK_TFLOPS, "traffic": None, "kernel": "k_update",
            "avg_launch_us": avg_s * 1e6, "flops_per_launch": flops_per_launch,
            "bytes_per_launch": g["bytes"] / g["launches"],
            "dominant_class": dom, "dominant_ms_per_step": prof[dom]["ms"] / max(steps, 1)}
