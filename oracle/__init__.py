"""CPU oracle for the tile Householder QR (test infrastructure only)."""
from .oracle import *  # noqa: F401,F403
from .oracle import build  # noqa: F401
