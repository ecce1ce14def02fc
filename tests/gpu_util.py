"""Helpers shared by the GPU tests (no method arithmetic here)."""
import sys
import time


def log(msg):
    sys.stdout.write("[%s] %s\n" % (time.strftime("%H:%M:%S"), msg))
    sys.stdout.flush()
