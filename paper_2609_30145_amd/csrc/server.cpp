// request server (added below)
