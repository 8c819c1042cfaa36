"""The named workloads of the benchmark and the kick-shape tuner: the seeded
synthetic systems of ``inputs`` under the names the measurements use."""
from __future__ import annotations

from . import inputs

DESCRIPTIONS = {
    "disk16k": "4 planets + 16384 planetesimals (m=1e-8, a~U[15,40], e~Rayleigh(0.05), "
               "i~Rayleigh(0.025)), tau=0.05, aE=3 mutual Hill radii, encounters on",
    "disk128k": "4 planets + 131072 planetesimals (m=2e-9, a~U[15,40], e~Rayleigh(0.05), "
                "i~Rayleigh(0.025)), tau=0.05, aE=3 mutual Hill radii, encounters on",
    "small": "4 planets + 100 planetesimals, tau=0.05",
    "batch": "512 systems, N~logU[64,4096]: 1 Jupiter-mass planet at 5.2 + planetesimals "
             "(m=1e-8, a~U[3,10]), tau=0.05, encounters on",
    "learned": "4 planets + 65536 planetesimals (m=1e-8, disk16k distributions, seed 6), "
               "tau=0.05, Kepler solve from the learned start (kepler_mode 2)",
}


def workload(name):
    """(list of systems, description) of a named workload."""
    if name == "disk16k":
        systems = [inputs.disk16k()]
    elif name == "disk128k":
        systems = [inputs.disk128k()]
    elif name == "small":
        systems = [inputs.small()]
    elif name == "batch":
        systems = inputs.batch()
    elif name == "learned":
        systems = [inputs.learned_workload(n_test=0)]
    else:
        raise ValueError(f"unknown workload {name}")
    return systems, DESCRIPTIONS[name]
