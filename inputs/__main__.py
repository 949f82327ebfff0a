"""python -m inputs geometry <workload> <path>: write a workload's geometry
file for native drivers (see write_geometry)."""
import sys

from . import write_geometry

if len(sys.argv) != 4 or sys.argv[1] != "geometry":
    sys.exit("usage: python -m inputs geometry <workload> <path>")
write_geometry(sys.argv[2], sys.argv[3])
