"""MI355X-native stochastic conservative field transfer (HIP, gfx950).

The HIP library ``libft.so`` (C ABI in ``include/ft.h``) is the product;
``ft`` is its ctypes binding.  Importing the package does not load the
library; ``ft.load()`` (or any ``ft.ft_*`` call) does, and fails loudly if it
has not been built.
"""
from . import ft  # noqa: F401

__all__ = ["ft"]
