"""Errors raised by the oracle (test infrastructure only)."""


class OracleError(RuntimeError):
    """Raised with a short code: EINVAL, ENOTSPD or ENONPOS_D."""

    def __init__(self, code: str, msg: str):
        super().__init__(f"{code}: {msg}")
        self.code = code
