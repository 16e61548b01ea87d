"""MI355X-native multigrid for high-order LDG systems (Poisson, elliptic
interface, multiphase Stokes): C-ABI library libldgmg.so and its binding."""
from . import ldgmg  # noqa: F401  (binding; loads the library on first use)
