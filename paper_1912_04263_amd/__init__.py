"""MI355X-native hot path of the GPU-accelerated OSQP-style ADMM (reduced-KKT PCG).

The compute path lives in the C-ABI library ``libqpg.so`` built from ``csrc/``;
``qpg`` is its thin ctypes binding. ``problems`` draws seeded synthetic inputs.
Importing the package loads nothing native; ``qpg`` loads the library on first
use and raises if it is missing.
"""
