"""MI355X-native quantum-walk step engine (coined and continuous-time walks).

The compute path is the HIP library ``libqwalk.so`` (C ABI in
``include/qwalk.h``); ``walk`` holds the torch-backed Python surface and
``inputs`` the seeded synthetic graph/state generators.  Importing this
package does not load the library; ``walk`` and ``_lib`` do, and fail loudly
if it is not built.
"""

__all__ = ["inputs", "walk", "build"]
