"""MI355X-native randomized QLP (RQLP / ERQLP / block RQLP)."""
from . import inputs  # noqa: F401
