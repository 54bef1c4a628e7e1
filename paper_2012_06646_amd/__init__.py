"""MI355X-native immersed-boundary spreading and interpolation.

Submodules:
    ibops      thin ctypes binding of the C-ABI library ``libibops.so`` (HIP kernels)
    workloads  seeded synthetic inputs (points, forces, grid fields, RBC surfaces)

Importing the package loads nothing; ``ibops`` loads the HIP library on import and raises
if it is missing.
"""
__version__ = "0.1.0"
